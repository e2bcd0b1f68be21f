// Diagnostics (Sec. 4, relative RMSE): sum (xa - xt)^2 and sum xt^2 over
// the observed quantity (u in 1D Burgers, rho u in 1D Euler, (u, v) =
// momentum/density in 2D) and the
// count of non-finite entries of xa.  Deterministic two-pass reduction in
// FP64: fixed per-block partials, then one block sums them in order.
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

__global__ __launch_bounds__(64) void diag_final(const double *__restrict__ part, int nblocks, double *__restrict__ out) {
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += part[3 * b + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

hipError_t launch_diagnostics(const Plan &p, const void *xa, const void *xt, double *out, void *ws, hipStream_t s) {
    double *part = (double *)((char *)ws + p.off_scratch);
    const long long nf = p.nf;
    // 1D: the observed field (u for Burgers, rho u for the Euler model)
    const size_t off = (size_t)p.obs_field * nf * p.tsize;
    xa = (const char *)xa + off;
    xt = (const char *)xt + off;
    int nb = (int)((nf + 255) / 256);
    if (nb > DIAG_BLOCKS) nb = DIAG_BLOCKS;
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(diag_partial<double>, dim3(nb), dim3(256), 0, s, (const double *)xa, (const double *)xt,
                           p.dim, nf, part);
    else
        hipLaunchKernelGGL(diag_partial<float>, dim3(nb), dim3(256), 0, s, (const float *)xa, (const float *)xt, p.dim,
                           nf, part);
    hipLaunchKernelGGL(diag_final, dim3(1), dim3(64), 0, s, (const double *)part, nb, out);
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

}  // namespace menkf
