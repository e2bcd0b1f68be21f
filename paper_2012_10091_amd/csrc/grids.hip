// Two-grid projections (Sec. 2.2): Pi_C (injection at the coincident nodes
// of nested vertex-centred periodic grids, which is what a fourth-order
// Lagrange restriction reduces to there) and Pi_F (four-point cubic
// Lagrange interpolation per direction, tensor product in 2D), plus the
// fine-grid correction x' = x^F_f + Pi_F(delta^C) of Algo. 4 step 5.
#include "common.hpp"

namespace menkf {

hipError_t launch_burgers_sweep(const Plan &p, const void *x, const void *xp, void *out, double alpha,
                                const int32_t *info, hipStream_t s);
hipError_t launch_ns_sweep(const Plan &p, const void *x, const void *xp, void *out, double alpha,
                           const int32_t *info, hipStream_t s);

template <typename T>
__global__ __launch_bounds__(256) void restrict_inject(const T *__restrict__ xf, T *__restrict__ xc, int nx,
                                                       int ny, int r, int nxc, int nyc, int F) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nc = (long long)nxc * nyc;
    if (i >= nc * F) return;
    const int f = (int)(i / nc);
    const long long j = i - f * nc;
    const int jy = (int)(j / nxc), jx = (int)(j - (long long)jy * nxc);
    xc[i] = xf[(long long)f * nx * ny + (long long)(jy * r) * nx + (long long)jx * r];
}

// xout = xin + Pi_F(dc) for every field; 1D when nyc == 1 (then ny == 1).
template <typename T>
__global__ __launch_bounds__(256) void prolong_add(const T *__restrict__ dc, const T *__restrict__ xin,
                                                   T *__restrict__ xout, int nx, int ny, int r, int nxc,
                                                   int nyc, int F, const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nf = (long long)nx * ny;
    if (i >= nf * F) return;
    const int f = (int)(i / nf);
    const long long j = i - f * nf;
    const int y = (int)(j / nx), x = (int)(j - (long long)y * nx);
    xout[i] = xin[i] + prolong_at<T>(dc + (long long)f * nxc * nyc, nxc, nyc, r, y, x);
}

// Open 1D grid (inlet-forced cases): xout = xin + Pi_F(dc) for every field
// with the one-sided cubic stencils of open_cubic, except at the inlet
// node, whose value the boundary condition prescribes (xout = xin there).
template <typename T>
__global__ __launch_bounds__(256) void prolong_add_open(const T *__restrict__ dc, const T *__restrict__ xin,
                                                        T *__restrict__ xout, int nx, int r, int nxc, int F,
                                                        const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nx * F) return;
    const int f = g / nx, x = g - f * nx;
    if (x == 0) {
        xout[g] = xin[g];
        return;
    }
    T w[4];
    const int b0 = open_cubic<T>(x, r, nxc, w);
    const T *d = dc + (long long)f * nxc;
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) acc += w[b] * d[b0 + b];
    xout[g] = xin[g] + acc;
}

// 2D form: one fine row of one field per grid row (y = blockIdx.y, field =
// blockIdx.z), so the coarse rows and y-weights are uniform per workgroup
// and the x-weights come from an LDS table of the r sub-positions.  Same
// weights and summation order as prolong_at.
template <typename T>
__global__ __launch_bounds__(256) void prolong_add_rows(const T *__restrict__ dc, const T *__restrict__ xin,
                                                        T *__restrict__ xout, int nx, int ny, int r, int nxc,
                                                        int nyc, const int32_t *__restrict__ info) {
    __shared__ T wxs[64][4];
    if (*info != 0) return;
    const int y = blockIdx.y, f = blockIdx.z;
    if ((int)threadIdx.x < r) lagrange4<T>(T(threadIdx.x) / T(r), wxs[threadIdx.x]);
    __syncthreads();
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    const int jy = y / r, my = y - jy * r;
    T wy[4];
    lagrange4<T>(T(my) / T(r), wy);
    const T *d = dc + (long long)f * nxc * nyc;
    const int jx = x / r, mx = x - jx * r;
    int cx[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        int v = jx - 1 + b;
        v += v < 0 ? nxc : 0;
        v -= v >= nxc ? nxc : 0;
        cx[b] = v;
    }
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const T *row = d + (long long)wrap(jy - 1 + a, nyc) * nxc;
        T sa = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) sa += wxs[mx][b] * row[cx[b]];
        acc += wy[a] * sa;
    }
    const long long g = ((long long)f * ny + y) * nx + x;
    xout[g] = xin[g] + acc;
}

// 2D form with the coarse rows staged: one workgroup per (fine row y,
// field); the four coarse rows jy - 1 .. jy + 2 under the row are read once
// into LDS (coalesced), then every fine point of the row interpolates from
// them.  Same weights and summation order (x first per coarse row, then
// y) as prolong_at, so the result is bitwise that of prolong_add_rows.
template <typename T>
__global__ __launch_bounds__(256) void prolong_add_staged(const T *__restrict__ dc, const T *__restrict__ xin,
                                                          T *__restrict__ xout, int nx, int ny, int r, int nxc,
                                                          int nyc, const int32_t *__restrict__ info) {
    extern __shared__ __align__(16) unsigned char smem_pa[];
    T(*wxs)[4] = reinterpret_cast<T(*)[4]>(smem_pa);          // [64][4]
    T *crow = reinterpret_cast<T *>(smem_pa + 64 * 4 * sizeof(T));   // [4][nxc]
    if (*info != 0) return;
    const int y = blockIdx.x, f = blockIdx.y;
    const int jy = y / r, my = y - jy * r;
    const T *d = dc + (long long)f * nxc * nyc;
    if ((int)threadIdx.x < r) lagrange4<T>(T(threadIdx.x) / T(r), wxs[threadIdx.x]);
    for (int e = threadIdx.x; e < 4 * nxc; e += 256) {
        const int a = e / nxc, j = e - a * nxc;
        int ry = jy - 1 + a;
        ry += ry < 0 ? nyc : 0;
        ry -= ry >= nyc ? nyc : 0;
        crow[e] = d[(long long)ry * nxc + j];
    }
    T wy[4];
    lagrange4<T>(T(my) / T(r), wy);
    __syncthreads();
    const long long g0 = ((long long)f * ny + y) * nx;
    for (int x = threadIdx.x; x < nx; x += 256) {
        const int jx = x / r, mx = x - jx * r;
        int cx[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int v = jx - 1 + b;
            v += v < 0 ? nxc : 0;
            v -= v >= nxc ? nxc : 0;
            cx[b] = v;
        }
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const T *row = crow + a * nxc;
            T sa = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) sa += wxs[mx][b] * row[cx[b]];
            acc += wy[a] * sa;
        }
        xout[g0 + x] = xin[g0 + x] + acc;
    }
}

// Members recentred on the injected fine state: one thread per coarse
// (field, point); the member mean is accumulated in FP64.
template <typename T>
__global__ __launch_bounds__(256) void recentre_members(T *__restrict__ X, const T *__restrict__ xf, int N,
                                                        long long npts, long long nc, long long nf, int nx, int r,
                                                        int nxc, const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const long long f = p / nc, q = p - f * nc;
    const long long jy = q / nxc, jx = q - jy * nxc;
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += (double)X[(long long)i * npts + p];
    const double shift = (double)xf[f * nf + (jy * r) * nx + jx * r] - s / (double)N;
    for (int i = 0; i < N; ++i) {
        T *v = X + (long long)i * npts + p;
        *v = (T)((double)*v + shift);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void copy_guarded(const T *__restrict__ src, T *__restrict__ dst, long long n,
                                                    const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_restrict(const Plan &p, const void *xf, void *xc, hipStream_t s) {
    const long long n = p.nc * p.F;
    const int blocks = (int)((n + 255) / 256);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(restrict_inject<double>, dim3(blocks), dim3(256), 0, s, (const double *)xf,
                           (double *)xc, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, p.F);
    else
        hipLaunchKernelGGL(restrict_inject<float>, dim3(blocks), dim3(256), 0, s, (const float *)xf,
                           (float *)xc, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, p.F);
    return hipGetLastError();
}

hipError_t launch_prolong_add(const Plan &p, const void *dc, const void *xin, void *xout, const int32_t *info,
                              hipStream_t s) {
    if (p.open) {
        const int blocks = (p.nx * p.F + 255) / 256;
        if (p.cfg.precision == MENKF_F64)
            hipLaunchKernelGGL(prolong_add_open<double>, dim3(blocks), dim3(256), 0, s, (const double *)dc,
                               (const double *)xin, (double *)xout, p.nx, p.cfg.ratio, p.nxc, p.F, info);
        else
            hipLaunchKernelGGL(prolong_add_open<float>, dim3(blocks), dim3(256), 0, s, (const float *)dc,
                               (const float *)xin, (float *)xout, p.nx, p.cfg.ratio, p.nxc, p.F, info);
        return hipGetLastError();
    }
    if (p.dim == 2 && p.cfg.ratio <= 64 && (size_t)(64 + p.nxc) * 4 * p.tsize <= 32768) {
        const dim3 grid(p.ny, p.F);
        const size_t lds = (size_t)(64 + p.nxc) * 4 * p.tsize;
        if (p.cfg.precision == MENKF_F64)
            hipLaunchKernelGGL(prolong_add_staged<double>, grid, dim3(256), lds, s, (const double *)dc,
                               (const double *)xin, (double *)xout, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, info);
        else
            hipLaunchKernelGGL(prolong_add_staged<float>, grid, dim3(256), lds, s, (const float *)dc,
                               (const float *)xin, (float *)xout, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, info);
        return hipGetLastError();
    }
    if (p.dim == 2 && p.ny <= 65535 && p.cfg.ratio <= 64) {
        const dim3 grid((p.nx + 255) / 256, p.ny, p.F);
        if (p.cfg.precision == MENKF_F64)
            hipLaunchKernelGGL(prolong_add_rows<double>, grid, dim3(256), 0, s, (const double *)dc,
                               (const double *)xin, (double *)xout, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, info);
        else
            hipLaunchKernelGGL(prolong_add_rows<float>, grid, dim3(256), 0, s, (const float *)dc,
                               (const float *)xin, (float *)xout, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, info);
        return hipGetLastError();
    }
    const long long n = p.nf * p.F;
    const int blocks = (int)((n + 255) / 256);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(prolong_add<double>, dim3(blocks), dim3(256), 0, s, (const double *)dc,
                           (const double *)xin, (double *)xout, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, p.F, info);
    else
        hipLaunchKernelGGL(prolong_add<float>, dim3(blocks), dim3(256), 0, s, (const float *)dc,
                           (const float *)xin, (float *)xout, p.nx, p.ny, p.cfg.ratio, p.nxc, p.nyc, p.F, info);
    return hipGetLastError();
}

hipError_t launch_recentre(const Plan &p, void *members, const void *xf, const int32_t *info, hipStream_t s) {
    const long long npts = p.nc * p.F;
    const int blocks = (int)((npts + 255) / 256);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(recentre_members<double>, dim3(blocks), dim3(256), 0, s, (double *)members,
                           (const double *)xf, p.N, npts, p.nc, p.nf, p.nx, p.cfg.ratio, p.nxc, info);
    else
        hipLaunchKernelGGL(recentre_members<float>, dim3(blocks), dim3(256), 0, s, (float *)members,
                           (const float *)xf, p.N, npts, p.nc, p.nf, p.nx, p.cfg.ratio, p.nxc, info);
    return hipGetLastError();
}

hipError_t launch_copy(const Plan &p, const void *src, void *dst, const int32_t *info, hipStream_t s) {
    const long long n = p.nf * p.F;
    const int blocks = (int)((n + 255) / 256);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(copy_guarded<double>, dim3(blocks), dim3(256), 0, s, (const double *)src,
                           (double *)dst, n, info);
    else
        hipLaunchKernelGGL(copy_guarded<float>, dim3(blocks), dim3(256), 0, s, (const float *)src, (float *)dst,
                           n, info);
    return hipGetLastError();
}

hipError_t launch_sweep(const Plan &p, const void *xin, const void *xprev, void *xout, double alpha,
                        const int32_t *info, void *ws, hipStream_t s) {
    (void)ws;
    if (p.cfg.model == MENKF_EULER1D_INLET) return launch_euler_sweep(p, xin, xprev, xout, alpha, info, s);
    if (p.dim == 1) return launch_burgers_sweep(p, xin, xprev, xout, alpha, info, s);
    return launch_ns_sweep(p, xin, xprev, xout, alpha, info, s);
}

}  // namespace menkf
