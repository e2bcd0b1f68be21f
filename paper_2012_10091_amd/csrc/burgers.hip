// 1D viscous Burgers forecast (Sec. 4, Burgers equation), advective form
// u_t = -u D1 u + nu D2 u with second-order centred differences on a
// periodic grid, advanced by the three-stage SSP Runge-Kutta scheme of
// Shu & Osher:
//   u1 = u + dt L(u);  u2 = 3/4 u + 1/4 (u1 + dt L(u1));  u' = 1/3 u + 2/3 (u2 + dt L(u2)).
//
// Two paths:
//  * window-in-LDS: one workgroup per member row, the row stays in LDS for
//    the whole observation window; HBM sees one read and one write per
//    window (plus the optional x_{k-1} copy).
//  * global stages: one launch per RK stage for rows too long for LDS.
#include "common.hpp"

namespace menkf {

template <typename T>
struct BurgersCoef {
    T dt, inv2h, nuih2;
};

template <typename T>
__device__ __forceinline__ T burgers_L(T um, T u, T up, const BurgersCoef<T> &c) {
    return -u * (up - um) * c.inv2h + c.nuih2 * (up - T(2) * u + um);
}

template <typename T, int PPT>
__global__ __launch_bounds__(1024) void burgers_window_lds(T *__restrict__ state, T *__restrict__ prev,
                                                           int n, int nsteps, BurgersCoef<T> c) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *P = reinterpret_cast<T *>(smem_raw);
    T *Q = P + n;
    const int bs = blockDim.x;
    T *row = state + (size_t)blockIdx.x * n;
    T *prow = prev ? prev + (size_t)blockIdx.x * n : nullptr;
    T u0[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = threadIdx.x + k * bs;
        if (i < n) {
            u0[k] = row[i];
            P[i] = u0[k];
        }
    }
    __syncthreads();
    for (int step = 0; step < nsteps; ++step) {
        if (prow && step == nsteps - 1) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = threadIdx.x + k * bs;
                if (i < n) prow[i] = u0[k];
            }
        }
        // stage 1: Q = u + dt L(P)   (P holds u)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = threadIdx.x + k * bs;
            if (i < n) {
                const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
                Q[i] = u0[k] + c.dt * burgers_L(P[im], P[i], P[ip], c);
            }
        }
        __syncthreads();
        // stage 2: P = 3/4 u + 1/4 (Q + dt L(Q))
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = threadIdx.x + k * bs;
            if (i < n) {
                const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
                const T q = Q[i];
                P[i] = T(0.75) * u0[k] + T(0.25) * (q + c.dt * burgers_L(Q[im], q, Q[ip], c));
            }
        }
        __syncthreads();
        // stage 3: Q = 1/3 u + 2/3 (P + dt L(P)) = new u
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = threadIdx.x + k * bs;
            if (i < n) {
                const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
                const T pp = P[i];
                const T un = u0[k] / T(3) + (T(2) / T(3)) * (pp + c.dt * burgers_L(P[im], pp, P[ip], c));
                u0[k] = un;
                Q[i] = un;
            }
        }
        __syncthreads();
        T *t = P;
        P = Q;
        Q = t;
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = threadIdx.x + k * bs;
        if (i < n) row[i] = u0[k];
    }
}

// One SSP-RK3 stage over global memory: out = a*u + b*(P + dt L(P)).
template <typename T>
__global__ __launch_bounds__(256) void burgers_stage(const T *__restrict__ Pin, const T *__restrict__ u,
                                                     T *__restrict__ out, T *__restrict__ prev, int n,
                                                     int nb, T a, T b, BurgersCoef<T> c) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)n * nb) return;
    const int i = (int)(gid % n);
    const long long base = gid - i;
    const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
    const T pp = Pin[gid];
    const T uu = u[gid];
    if (prev) prev[gid] = uu;
    out[gid] = a * uu + b * (pp + c.dt * burgers_L(Pin[base + im], pp, Pin[base + ip], c));
}

// Relaxed Jacobi sweep of x - dt L(x) = x_prev:  x' = x + w (x_prev + dt L(x) - x),  w = alpha / D.
template <typename T>
__global__ __launch_bounds__(256) void burgers_sweep(const T *__restrict__ x, const T *__restrict__ xp,
                                                     T *__restrict__ out, int n, T w, BurgersCoef<T> c,
                                                     const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
    const T xx = x[i];
    out[i] = xx + w * (xp[i] + c.dt * burgers_L(x[im], xx, x[ip], c) - xx);
}

// Implicit-Euler residual r = x_prev + dt L(x) - x.
template <typename T>
__global__ __launch_bounds__(256) void burgers_resid(const T *__restrict__ x, const T *__restrict__ xp,
                                                     T *__restrict__ out, int n, BurgersCoef<T> c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
    const T xx = x[i];
    out[i] = xp[i] + c.dt * burgers_L(x[im], xx, x[ip], c) - xx;
}

// ----------------------------------------------------------------- inlet-forced case
// Open grid, nodes x_i = i h (Sec. 4 inlet case): Dirichlet inlet
// u(0, t) = u0 (1 + th0 sin(omega t + th1)) with the parameters th of the
// state's own row, imposed at every stage time (t + dt, t + dt/2, t + dt);
// the outlet node is the linear extrapolation 2 u_{n-2} - u_{n-3} of each
// stage's interior values.  One workgroup per state; the step-start state U
// and the two stage arrays stay in LDS for the whole window.  The thread
// that owns the outlet node recomputes the two interior values it
// extrapolates from (they are read from the stage's inputs only, so no
// extra barrier is needed).  Inlet values of up to GCH steps at a time are
// tabulated in LDS by all threads together before they are needed.
constexpr int INLET_GCH = 256;

template <typename T>
struct InletCoef {
    double u0, omega, dt;   // the boundary value is evaluated in FP64
};

template <int S, typename T>
__device__ __forceinline__ T inlet_stage_val(const T *__restrict__ U, const T *__restrict__ X, int i,
                                             const BurgersCoef<T> &c) {
    const T xi = X[i];
    const T v = xi + c.dt * burgers_L(X[i - 1], xi, X[i + 1], c);
    if (S == 1) return v;
    if (S == 2) return T(0.75) * U[i] + T(0.25) * v;
    return U[i] / T(3) + (T(2) / T(3)) * v;
}

template <int S, int PPT, typename T>
__device__ __forceinline__ void inlet_stage(const T *__restrict__ U, const T *__restrict__ X, T *__restrict__ Y,
                                            int n, T g, const BurgersCoef<T> &c) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = threadIdx.x + k * blockDim.x;
        if (i >= n) continue;
        T v;
        if (i == 0)
            v = g;
        else if (i < n - 1)
            v = inlet_stage_val<S>(U, X, i, c);
        else
            v = T(2) * inlet_stage_val<S>(U, X, n - 2, c) - inlet_stage_val<S>(U, X, n - 3, c);
        Y[i] = v;
    }
}

// SCHEME 0: three-stage SSP-RK3 steps.  SCHEME 1: the paper's first-order
// scheme: forward-Euler steps, and the window's last step (the analysis
// step) as one Jacobi iteration of the implicit-Euler system from x_{k-1},
// x_k = x_{k-1} + (dt / D) L(x_{k-1}), D = 1 + 2 nu dt / h^2 (coefficients
// cj, whose dt is dt / D).
template <typename T, int PPT, int SCHEME>
__global__ __launch_bounds__(1024) void burgers_inlet_window(T *__restrict__ state, T *__restrict__ prev, int n,
                                                             int nsteps, BurgersCoef<T> c, BurgersCoef<T> cj,
                                                             InletCoef<T> ic, const double *__restrict__ theta,
                                                             const double *__restrict__ t0p) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *G = reinterpret_cast<T *>(smem_raw);   // [INLET_GCH][2]: g(t + dt), g(t + dt/2)
    T *U = G + 2 * INLET_GCH;
    T *A = U + n;
    T *B = A + n;
    const int bs = blockDim.x;
    T *row = state + (size_t)blockIdx.x * n;
    T *prow = prev ? prev + (size_t)blockIdx.x * n : nullptr;
    const double th0 = theta[2 * blockIdx.x], th1 = theta[2 * blockIdx.x + 1];
    const double t0 = *t0p;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = threadIdx.x + k * bs;
        if (i < n) U[i] = row[i];
    }
    for (int base = 0; base < nsteps; base += INLET_GCH) {
        const int cnt = nsteps - base < INLET_GCH ? nsteps - base : INLET_GCH;
        __syncthreads();   // the previous chunk's table is no longer read
        for (int q = threadIdx.x; q < 2 * cnt; q += bs) {
            const double tt = t0 + (double)(base + (q >> 1)) * ic.dt;
            const double ts = (q & 1) ? tt + 0.5 * ic.dt : tt + ic.dt;
            G[q] = (T)(ic.u0 * (1.0 + th0 * sin(ic.omega * ts + th1)));
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const int step = base + j;
            if (prow && step == nsteps - 1) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int i = threadIdx.x + k * bs;
                    if (i < n) prow[i] = U[i];
                }
            }
            const T g1 = G[2 * j], g2 = G[2 * j + 1];
            if (SCHEME == 1) {
                inlet_stage<1, PPT>(U, U, A, n, g1, step == nsteps - 1 ? cj : c);   // the new state, into A
                __syncthreads();
            } else {
                inlet_stage<1, PPT>(U, U, A, n, g1, c);
                __syncthreads();
                inlet_stage<2, PPT>(U, A, B, n, g2, c);
                __syncthreads();
                inlet_stage<3, PPT>(U, B, A, n, g1, c);   // the new state, into A
                __syncthreads();
            }
            T *t = U;
            U = A;
            A = t;
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = threadIdx.x + k * bs;
        if (i < n) row[i] = U[i];
    }
}

// Relaxed Jacobi sweep on the open grid: interior as in the periodic case,
// the inlet node kept, the outlet extrapolated from the swept interior.
template <typename T>
__device__ __forceinline__ T sweep_val(const T *__restrict__ x, const T *__restrict__ xp, int i, T w,
                                       const BurgersCoef<T> &c) {
    const T xx = x[i];
    return xx + w * (xp[i] + c.dt * burgers_L(x[i - 1], xx, x[i + 1], c) - xx);
}

template <typename T>
__global__ __launch_bounds__(256) void burgers_sweep_inlet(const T *__restrict__ x, const T *__restrict__ xp,
                                                           T *__restrict__ out, int n, T w, BurgersCoef<T> c,
                                                           const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T v;
    if (i == 0)
        v = x[0];
    else if (i < n - 1)
        v = sweep_val(x, xp, i, w, c);
    else
        v = T(2) * sweep_val(x, xp, n - 2, w, c) - sweep_val(x, xp, n - 3, w, c);
    out[i] = v;
}

template <typename T>
static BurgersCoef<T> make_coef(const Plan &p, int level) {
    const int n = level == MENKF_FINE ? p.nx : p.nxc;
    const double h = p.cfg.length / n;
    BurgersCoef<T> c;
    c.dt = (T)p.cfg.dt;
    c.inv2h = (T)(1.0 / (2.0 * h));
    c.nuih2 = (T)(p.cfg.nu / (h * h));
    return c;
}

template <typename T, int PPT>
static hipError_t launch_window(T *state, T *prev, int n, int nb, int nsteps, BurgersCoef<T> c, int bs,
                                hipStream_t s) {
    const size_t lds = 2 * (size_t)n * sizeof(T);
    auto kern = burgers_window_lds<T, PPT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, s, state, prev, n, nsteps, c);
    return hipGetLastError();
}

template <typename T>
static hipError_t burgers_forecast_t(const Plan &p, int level, T *state, int nb, int nsteps, T *prev,
                                     void *ws, hipStream_t s) {
    const int n = level == MENKF_FINE ? p.nx : p.nxc;
    const BurgersCoef<T> c = make_coef<T>(p, level);
    const size_t lds = 2 * (size_t)n * sizeof(T);
    if (lds <= 128 * 1024) {
        int bs = 64;
        while (bs < 1024 && bs < n) bs *= 2;
        const int ppt = (n + bs - 1) / bs;
        if (ppt <= 1) return launch_window<T, 1>(state, prev, n, nb, nsteps, c, bs, s);
        if (ppt <= 2) return launch_window<T, 2>(state, prev, n, nb, nsteps, c, bs, s);
        if (ppt <= 4) return launch_window<T, 4>(state, prev, n, nb, nsteps, c, bs, s);
        if (ppt <= 8) return launch_window<T, 8>(state, prev, n, nb, nsteps, c, bs, s);
        if (ppt <= 16) return launch_window<T, 16>(state, prev, n, nb, nsteps, c, bs, s);
        if (ppt <= 32) return launch_window<T, 32>(state, prev, n, nb, nsteps, c, bs, s);
    }
    // global-memory stages
    char *w = (char *)ws;
    T *s1 = (T *)(w + (level == MENKF_FINE ? p.off_f1 : p.off_c1));
    T *s2 = (T *)(w + (level == MENKF_FINE ? p.off_f2 : p.off_c2));
    const long long tot = (long long)n * nb;
    const int blocks = (int)((tot + 255) / 256);
    for (int step = 0; step < nsteps; ++step) {
        T *pv = (prev && step == nsteps - 1) ? prev : nullptr;
        hipLaunchKernelGGL(burgers_stage<T>, dim3(blocks), dim3(256), 0, s, state, state, s1, pv, n, nb,
                           T(0), T(1), c);
        hipLaunchKernelGGL(burgers_stage<T>, dim3(blocks), dim3(256), 0, s, s1, state, s2, (T *)nullptr, n, nb,
                           T(0.75), T(0.25), c);
        hipLaunchKernelGGL(burgers_stage<T>, dim3(blocks), dim3(256), 0, s, s2, state, state, (T *)nullptr, n,
                           nb, T(1) / T(3), T(2) / T(3), c);
    }
    return hipGetLastError();
}

size_t inlet_window_lds(int n, size_t tsize) { return (2 * (size_t)INLET_GCH + 3 * (size_t)n) * tsize; }

template <typename T, int PPT>
static hipError_t launch_inlet(T *state, T *prev, int n, int nb, int nsteps, BurgersCoef<T> c, BurgersCoef<T> cj,
                               InletCoef<T> ic, int scheme, const double *theta, const double *t0, int bs,
                               hipStream_t s) {
    const size_t lds = inlet_window_lds(n, sizeof(T));
    auto kern = scheme == MENKF_TIME_FIRST_ORDER ? burgers_inlet_window<T, PPT, 1> : burgers_inlet_window<T, PPT, 0>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, s, state, prev, n, nsteps, c, cj, ic, theta, t0);
    return hipGetLastError();
}

template <typename T>
static hipError_t inlet_forecast_t(const Plan &p, int level, T *state, int nb, int nsteps, T *prev,
                                   const double *theta, const double *t0, hipStream_t s) {
    const int n = level == MENKF_FINE ? p.nx : p.nxc;
    const BurgersCoef<T> c = make_coef<T>(p, level);
    // the Jacobi iteration of the analysis step: dt scaled by 1/D, D the
    // diagonal 1 + 2 nu dt / h^2 of the implicit-Euler matrix on this level
    BurgersCoef<T> cj = c;
    const double h = p.cfg.length / n;
    cj.dt = (T)(p.cfg.dt / (1.0 + 2.0 * p.cfg.nu * p.cfg.dt / (h * h)));
    const int sch = p.cfg.time_scheme;
    const InletCoef<T> ic{p.cfg.u0, p.cfg.omega, p.cfg.dt};
    int bs = 64;
    while (bs < 1024 && bs < n) bs *= 2;
    const int ppt = (n + bs - 1) / bs;
    if (ppt <= 1) return launch_inlet<T, 1>(state, prev, n, nb, nsteps, c, cj, ic, sch, theta, t0, bs, s);
    if (ppt <= 2) return launch_inlet<T, 2>(state, prev, n, nb, nsteps, c, cj, ic, sch, theta, t0, bs, s);
    if (ppt <= 4) return launch_inlet<T, 4>(state, prev, n, nb, nsteps, c, cj, ic, sch, theta, t0, bs, s);
    if (ppt <= 8) return launch_inlet<T, 8>(state, prev, n, nb, nsteps, c, cj, ic, sch, theta, t0, bs, s);
    return hipErrorInvalidValue;   // rows this long are rejected when the context is created
}

hipError_t launch_inlet_forecast(const Plan &p, int level, void *state, int nb, int nsteps, void *prev,
                                 const double *theta, const double *t0, hipStream_t s) {
    if (p.cfg.model == MENKF_EULER1D_INLET) return launch_euler_forecast(p, level, state, nb, nsteps, prev, theta, t0, s);
    if (p.cfg.precision == MENKF_F64)
        return inlet_forecast_t<double>(p, level, (double *)state, nb, nsteps, (double *)prev, theta, t0, s);
    return inlet_forecast_t<float>(p, level, (float *)state, nb, nsteps, (float *)prev, theta, t0, s);
}

hipError_t launch_burgers_forecast(const Plan &p, int level, void *state, int nb, int nsteps, void *prev,
                                   void *ws, hipStream_t s) {
    if (p.cfg.precision == MENKF_F64)
        return burgers_forecast_t<double>(p, level, (double *)state, nb, nsteps, (double *)prev, ws, s);
    return burgers_forecast_t<float>(p, level, (float *)state, nb, nsteps, (float *)prev, ws, s);
}

template <typename T>
static hipError_t burgers_sweep_t(const Plan &p, const T *x, const T *xp, T *out, double alpha,
                                  const int32_t *info, hipStream_t s) {
    const BurgersCoef<T> c = make_coef<T>(p, MENKF_FINE);
    const double h = p.cfg.length / p.nx;
    const double D = 1.0 + p.cfg.dt * p.cfg.nu * 2.0 / (h * h);
    if (p.open)
        hipLaunchKernelGGL(burgers_sweep_inlet<T>, dim3((p.nx + 255) / 256), dim3(256), 0, s, x, xp, out, p.nx,
                           (T)(alpha / D), c, info);
    else
        hipLaunchKernelGGL(burgers_sweep<T>, dim3((p.nx + 255) / 256), dim3(256), 0, s, x, xp, out, p.nx,
                           (T)(alpha / D), c, info);
    return hipGetLastError();
}

hipError_t launch_burgers_sweep(const Plan &p, const void *x, const void *xp, void *out, double alpha,
                                const int32_t *info, hipStream_t s) {
    if (p.cfg.precision == MENKF_F64)
        return burgers_sweep_t<double>(p, (const double *)x, (const double *)xp, (double *)out, alpha, info, s);
    return burgers_sweep_t<float>(p, (const float *)x, (const float *)xp, (float *)out, alpha, info, s);
}

hipError_t launch_burgers_resid(const Plan &p, const void *x, const void *xp, void *out, hipStream_t s) {
    const int blocks = (p.nx + 255) / 256;
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(burgers_resid<double>, dim3(blocks), dim3(256), 0, s, (const double *)x, (const double *)xp,
                           (double *)out, p.nx, make_coef<double>(p, MENKF_FINE));
    else
        hipLaunchKernelGGL(burgers_resid<float>, dim3(blocks), dim3(256), 0, s, (const float *)x, (const float *)xp,
                           (float *)out, p.nx, make_coef<float>(p, MENKF_FINE));
    return hipGetLastError();
}

}  // namespace menkf
