// Dual EnKF parameter filter (Sec. 2.1.3, Algo. 2) of the inlet-forced
// case: random-walk forecast of the members' parameters, their ensemble
// Kalman update with the gain factors of the preceding analysis, and the
// clock of the dual cycle.
#include "common.hpp"

namespace menkf {

constexpr int DUAL_P = 2;   // (amplitude, phase) of the inlet forcing

// theta_f[i][k] = theta[i][k] + sigma_k z, z the standard normal of Philox
// stream 0x5041 at counter (k >> 1, i, cycle); the cycle comes from the
// device counter when dcycle is given (read, not advanced).
__global__ __launch_bounds__(256) void param_perturb(const double *__restrict__ theta, double *__restrict__ thf,
                                                     int N, double s0, double s1, uint64_t seed, uint64_t cycle,
                                                     const uint64_t *__restrict__ dcycle) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N * DUAL_P) return;
    if (dcycle) cycle = *dcycle;
    const int i = q / DUAL_P, k = q - i * DUAL_P;
    thf[q] = theta[q] + (k == 0 ? s0 : s1) * philox_normal(seed, cycle, i, k, 0x5041u);
}

// theta_a(j) = theta_f(j) + sum_i Theta_i Z[i, j] (Algo. 2 step 5), Theta the
// parameter anomalies (theta_f(i) - mean) / sqrt(N - 1); Z[i, j] is stored at
// z[j N + i].  theta_a may alias theta_f (read into LDS first).  tmean gets
// the mean of theta_a.  One workgroup, FP64; a no-op if the status is set.
__global__ __launch_bounds__(256) void param_update(const double *__restrict__ thf, double *__restrict__ tha,
                                                    double *__restrict__ tmean, const double *__restrict__ z, int N,
                                                    const int32_t *__restrict__ info) {
    __shared__ double s_th[256][DUAL_P];
    __shared__ double s_new[256][DUAL_P];
    __shared__ double s_mean[DUAL_P];
    if (*info != 0) return;
    const int t = threadIdx.x;
    if (t < N)
        for (int k = 0; k < DUAL_P; ++k) s_th[t][k] = thf[t * DUAL_P + k];
    __syncthreads();
    if (t < DUAL_P) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += s_th[i][t];
        s_mean[t] = acc / (double)N;
    }
    __syncthreads();
    const double inv = 1.0 / sqrt((double)(N - 1));
    if (t < N) {
        const double *zc = z + (size_t)t * N;
        for (int k = 0; k < DUAL_P; ++k) {
            double acc = 0.0;
            for (int i = 0; i < N; ++i) acc += (s_th[i][k] - s_mean[k]) * inv * zc[i];
            s_new[t][k] = s_th[t][k] + acc;
            tha[t * DUAL_P + k] = s_new[t][k];
        }
    }
    __syncthreads();
    if (t < DUAL_P) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += s_new[i][t];
        tmean[t] = acc / (double)N;
    }
}

__global__ void clock_advance(double *clock, double dt_window) {
    if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] = clock[0] + dt_window;
}

// Start of a dual cycle in one launch: the trial copy of the members (the
// parameter filter forecasts them with theta_f) and theta_f itself.
template <typename T>
__global__ __launch_bounds__(256) void dual_prep(const T *__restrict__ members, T *__restrict__ trial, long long n,
                                                 const double *__restrict__ theta, double *__restrict__ thf, int N,
                                                 double s0, double s1, uint64_t seed, uint64_t cycle,
                                                 const uint64_t *__restrict__ dcycle) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) trial[q] = members[q];
    if (q < (long long)N * DUAL_P) {
        if (dcycle) cycle = *dcycle;
        const int i = (int)q / DUAL_P, k = (int)q - i * DUAL_P;
        thf[q] = theta[q] + (k == 0 ? s0 : s1) * philox_normal(seed, cycle, i, k, 0x5041u);
    }
}

hipError_t launch_dual_prep(const Plan &p, const void *members, void *trial, const double *theta, double *thf,
                            uint64_t seed, uint64_t cycle, void *ws, hipStream_t s) {
    const uint64_t *dcycle =
        cycle == MENKF_CYCLE_DEVICE ? (const uint64_t *)((char *)ws + p.off_info + 64) : nullptr;
    const long long n = (long long)p.N * p.nc * p.F;
    const long long work = n > (long long)p.N * DUAL_P ? n : (long long)p.N * DUAL_P;
    const dim3 grid((unsigned)((work + 255) / 256));
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(dual_prep<double>, grid, dim3(256), 0, s, (const double *)members, (double *)trial, n, theta,
                           thf, p.N, p.cfg.theta_sigma[0], p.cfg.theta_sigma[1], seed, cycle, dcycle);
    else
        hipLaunchKernelGGL(dual_prep<float>, grid, dim3(256), 0, s, (const float *)members, (float *)trial, n, theta,
                           thf, p.N, p.cfg.theta_sigma[0], p.cfg.theta_sigma[1], seed, cycle, dcycle);
    return hipGetLastError();
}

hipError_t launch_param_perturb(const Plan &p, const double *theta, double *thf, uint64_t seed, uint64_t cycle,
                                void *ws, hipStream_t s) {
    const uint64_t *dcycle =
        cycle == MENKF_CYCLE_DEVICE ? (const uint64_t *)((char *)ws + p.off_info + 64) : nullptr;
    const int n = p.N * DUAL_P;
    hipLaunchKernelGGL(param_perturb, dim3((n + 255) / 256), dim3(256), 0, s, theta, thf, p.N, p.cfg.theta_sigma[0],
                       p.cfg.theta_sigma[1], seed, cycle, dcycle);
    return hipGetLastError();
}

hipError_t launch_param_update(const Plan &p, const double *thf, double *tha, double *tmean, void *ws,
                               hipStream_t s) {
    char *w = (char *)ws;
    hipLaunchKernelGGL(param_update, dim3(1), dim3(256), 0, s, thf, tha, tmean, (const double *)(w + p.off_z), p.N,
                       (const int32_t *)(w + p.off_info));
    return hipGetLastError();
}

hipError_t launch_clock_advance(double *clock, double dt_window, hipStream_t s) {
    hipLaunchKernelGGL(clock_advance, dim3(1), dim3(64), 0, s, clock, dt_window);
    return hipGetLastError();
}

}  // namespace menkf
