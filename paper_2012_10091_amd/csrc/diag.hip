// Diagnostics (Sec. 4, relative RMSE): sum (xa - xt)^2 and sum xt^2 over
// the observed quantity (u in 1D Burgers, rho u in 1D Euler, (u, v) =
// momentum/density in 2D) and the count of non-finite entries of xa; and
// the ensemble spread: the trace of the ensemble error covariance
// P^e = X X^T (Sec. 2.1.2) over the same quantity of the coarse members,
// with the squared ensemble mean for its normalisation.  Deterministic
// two-pass reductions in FP64: fixed per-block partials, then one block
// sums them in order.
#include <mutex>

#include "common.hpp"

namespace menkf {

constexpr int DIAG_BLOCKS = 512;

template <typename T>
__global__ __launch_bounds__(256) void diag_partial(const T *__restrict__ xa, const T *__restrict__ xt, int dim,
                                                    long long nf, double *__restrict__ part) {
    __shared__ double s0[256], s1[256], s2[256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < nf; i += (long long)gridDim.x * 256) {
        if (dim == 1) {
            const double va = (double)xa[i], vt = (double)xt[i];
            if (!isfinite(va)) c += 1.0;
            a += (va - vt) * (va - vt);
            b += vt * vt;
        } else {
            const double ra = (double)xa[i], rt = (double)xt[i];
            const double ua = (double)xa[nf + i] / ra, va = (double)xa[2 * nf + i] / ra;
            const double ut = (double)xt[nf + i] / rt, vt = (double)xt[2 * nf + i] / rt;
            for (int f = 0; f < 4; ++f)
                if (!isfinite((double)xa[f * nf + i])) c += 1.0;
            a += (ua - ut) * (ua - ut) + (va - vt) * (va - vt);
            b += ut * ut + vt * vt;
        }
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s0[0];
        part[3 * blockIdx.x + 1] = s1[0];
        part[3 * blockIdx.x + 2] = s2[0];
    }
}

// Ensemble spread, one grid point per thread and loop: the members' values
// q^(k) of the observed quantity are summed as deviations from the first
// member's value (shifted sums s1 = sum d, s2 = sum d^2, d = q^(k) - q^(0)),
// so sum_k (q^(k) - mean)^2 = s2 - s1^2 / nb and mean = q^(0) + s1 / nb
// carry no cancellation of the mean's magnitude.  A single pass over the
// members, all in FP64.
template <typename T>
__global__ __launch_bounds__(256) void spread_partial(const T *__restrict__ mem, int dim, long long nc,
                                                      long long mstride, int nb, double inv_nm1,
                                                      double *__restrict__ part) {
    __shared__ double s0[256], s1[256], s2[256];
    double a = 0.0, b = 0.0, c = 0.0;
    const double inv_nb = 1.0 / (double)nb;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < nc; i += (long long)gridDim.x * 256) {
        if (dim == 1) {
            const double q0 = (double)mem[i];
            double su = 0.0, sq = 0.0;
            for (int k = 0; k < nb; ++k) {
                const double q = (double)mem[k * mstride + i];
                if (!isfinite(q)) c += 1.0;
                const double d = q - q0;
                su += d;
                sq += d * d;
            }
            a += (sq - su * su * inv_nb) * inv_nm1;
            const double mean = q0 + su * inv_nb;
            b += mean * mean;
        } else {
            const double u0 = (double)mem[nc + i] / (double)mem[i];
            const double v0 = (double)mem[2 * nc + i] / (double)mem[i];
            double su = 0.0, squ = 0.0, sv = 0.0, sqv = 0.0;
            for (int k = 0; k < nb; ++k) {
                const T *mk = mem + k * mstride;
                const double r = (double)mk[i];
                const double u = (double)mk[nc + i] / r, v = (double)mk[2 * nc + i] / r;
                if (!isfinite(u)) c += 1.0;
                if (!isfinite(v)) c += 1.0;
                const double du = u - u0, dv = v - v0;
                su += du;
                squ += du * du;
                sv += dv;
                sqv += dv * dv;
            }
            a += ((squ - su * su * inv_nb) + (sqv - sv * sv * inv_nb)) * inv_nm1;
            const double mu = u0 + su * inv_nb, mv = v0 + sv * inv_nb;
            b += mu * mu + mv * mv;
        }
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s0[0];
        part[3 * blockIdx.x + 1] = s1[0];
        part[3 * blockIdx.x + 2] = s2[0];
    }
}

// Sum of the per-block partials in a fixed order: thread t adds partials
// t, t + 256, ... of each quantity, then a tree over the 256 threads.
__global__ __launch_bounds__(256) void diag_final(const double *__restrict__ part, int nblocks, double *__restrict__ out) {
    __shared__ double s[3][256];
    double a[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
        for (int q = 0; q < 3; ++q) a[q] += part[3 * b + q];
    for (int q = 0; q < 3; ++q) s[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = s[threadIdx.x][0];
}

// Number of reduction workgroups of the diagnostics (each writes three partials).
static int diagnostics_blocks(const Plan &p) {
    const long long nb = (p.nf + 255) / 256;
    return nb > DIAG_BLOCKS ? DIAG_BLOCKS : (int)nb;
}

static hipError_t diagnostics_into(const Plan &p, const void *xa, const void *xt, double *out, double *part,
                                   hipStream_t s) {
    const long long nf = p.nf;
    // 1D: the observed field (u for Burgers, rho u for the Euler model)
    const size_t off = (size_t)p.obs_field * nf * p.tsize;
    xa = (const char *)xa + off;
    xt = (const char *)xt + off;
    const int nb = diagnostics_blocks(p);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(diag_partial<double>, dim3(nb), dim3(256), 0, s, (const double *)xa, (const double *)xt,
                           p.dim, nf, part);
    else
        hipLaunchKernelGGL(diag_partial<float>, dim3(nb), dim3(256), 0, s, (const float *)xa, (const float *)xt, p.dim,
                           nf, part);
    hipLaunchKernelGGL(diag_final, dim3(1), dim3(256), 0, s, (const double *)part, nb, out);
    return hipGetLastError();
}

hipError_t launch_diagnostics(const Plan &p, const void *xa, const void *xt, double *out, void *ws, hipStream_t s) {
    return diagnostics_into(p, xa, xt, out, (double *)((char *)ws + p.off_scratch), s);
}

// Reduction partials of the allocation-free diagnostics: a fixed device
// array in place of the context workspace.  Every device the library runs
// on holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device (the
// array's name in host code is not a device address).
constexpr int NOALLOC_DOUBLES = 2048;   // 16 KiB: room for 682 workgroups' partials
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// The scratch array's address on the current device, looked up once per
// device (with that device current) and kept.
static hipError_t noalloc_scratch(double **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        double *a = nullptr;
        e = hipGetSymbolAddress((void **)&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = a;
    }
    *ptr = g_scratch_dev[dev];
    return hipSuccess;
}

size_t diagnostics_noalloc_need(const Plan &p) { return (size_t)3 * diagnostics_blocks(p); }
size_t diagnostics_noalloc_capacity() { return NOALLOC_DOUBLES; }

// Every partial the final sum reads is written by the same call first, so
// the array needs no clearing between calls.
hipError_t launch_diagnostics_noalloc(const Plan &p, const void *xa, const void *xt, double *out, hipStream_t s) {
    double *part = nullptr;
    const hipError_t e = noalloc_scratch(&part);
    if (e != hipSuccess) return e;
    return diagnostics_into(p, xa, xt, out, part, s);
}

hipError_t launch_spread(const Plan &p, const void *members, int nb, double *out, void *ws, hipStream_t s) {
    double *part = (double *)((char *)ws + p.off_scratch);
    const long long nc = p.nc;
    const long long mstride = (long long)p.F * nc;
    // 1D: the observed field of every member (u for Burgers, rho u for Euler)
    const size_t off = (size_t)p.obs_field * nc * p.tsize;
    const void *m = (const char *)members + (p.dim == 1 ? off : 0);
    int nblk = (int)((nc + 255) / 256);
    if (nblk > DIAG_BLOCKS) nblk = DIAG_BLOCKS;
    const double inv_nm1 = 1.0 / (double)(nb - 1);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(spread_partial<double>, dim3(nblk), dim3(256), 0, s, (const double *)m, p.dim, nc, mstride,
                           nb, inv_nm1, part);
    else
        hipLaunchKernelGGL(spread_partial<float>, dim3(nblk), dim3(256), 0, s, (const float *)m, p.dim, nc, mstride,
                           nb, inv_nm1, part);
    hipLaunchKernelGGL(diag_final, dim3(1), dim3(256), 0, s, (const double *)part, nblk, out);
    return hipGetLastError();
}

__global__ void set_word(int32_t *w, int32_t v) { *w = v; }
__global__ void set_word64(uint64_t *w, uint64_t v) { *w = v; }

hipError_t launch_set_word(int32_t *w, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(set_word, dim3(1), dim3(1), 0, s, w, v);
    return hipGetLastError();
}

hipError_t launch_set_word64(uint64_t *w, uint64_t v, hipStream_t s) {
    hipLaunchKernelGGL(set_word64, dim3(1), dim3(1), 0, s, w, v);
    return hipGetLastError();
}

// skip word of a deferred correction: nothing pending, or a failed analysis
__global__ void pipe_skip_kernel(const int32_t *__restrict__ info, int32_t *__restrict__ pw) {
    pw[PW_SKIP] = (pw[PW_PEND] == 0 || *info != 0) ? 1 : 0;
}

hipError_t launch_pipe_skip(const int32_t *info, int32_t *pw, hipStream_t s) {
    hipLaunchKernelGGL(pipe_skip_kernel, dim3(1), dim3(1), 0, s, info, pw);
    return hipGetLastError();
}

}  // namespace menkf
