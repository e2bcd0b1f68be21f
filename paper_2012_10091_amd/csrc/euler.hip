// Inviscid 1D Euler equations of the acoustic-wave case (Sec. 5), inlet
// forced, in conservative variables (rho, rho u, rho E), characteristic
// units (u0 + a = 1, rho0 = 1): second-order centred flux differences,
// forward Euler in time (the single matrix-splitting iteration of an
// analysis step, started from x_{k-1}, is that same step: the centred
// inviscid operator has no diagonal), and a centred explicit filter of
// order 6 on nodes 3..n-4, 4 on nodes 2 and n-3, 2 on nodes 1 and n-2,
//   x <- x + (-1)^(p+1) sigma delta^(2p) x / 4^p   (transfer 1 - sigma sin^(2p)(k h / 2)).
// One step: interior update, inlet state (rho0, rho0 u_in(t + dt), rho0 E0)
// with u_in = u0 (1 + theta_1 sin(omega t + theta_2)), filter, outlet node
// extrapolated linearly from the two before it.
#include "common.hpp"

namespace menkf {

template <typename T>
struct EulerCoef {
    T dt, inv2h, gm1, sig;      // dt, 1/(2h), gamma - 1, filter strength
    T rho0, e0;                 // inlet density and total energy density rho0 E0
    double u0, omega, dtd;      // inlet velocity law, evaluated in FP64
};

template <typename T>
__device__ __forceinline__ void euler_flux(T rho, T m, T e, T gm1, T &f0, T &f1, T &f2) {
    const T u = m / rho;
    const T p = gm1 * (e - T(0.5) * m * u);
    f0 = m;
    f1 = m * u + p;
    f2 = (e + p) * u;
}

// Filtered value at node i of field row Y (n nodes, 1 <= i <= n-2).
template <typename T>
__device__ __forceinline__ T euler_filter_at(const T *__restrict__ Y, int i, int n, T sig) {
    const T y = Y[i];
    if (i >= 3 && i <= n - 4) {
        const T d = (Y[i - 3] + Y[i + 3]) - T(6) * (Y[i - 2] + Y[i + 2]) + T(15) * (Y[i - 1] + Y[i + 1]) - T(20) * y;
        return y + sig * d * T(1.0 / 64.0);
    }
    if (i == 2 || i == n - 3) {
        const T d = (Y[i - 2] + Y[i + 2]) - T(4) * (Y[i - 1] + Y[i + 1]) + T(6) * y;
        return y - sig * d * T(1.0 / 16.0);
    }
    const T d = (Y[i - 1] + Y[i + 1]) - T(2) * y;
    return y + sig * d * T(0.25);
}

constexpr int EULER_GCH = 256;

// One workgroup per state.  LDS: X (state, 3 rows), Y (updated, before the
// filter), Fl (fluxes of X), G (inlet momentum of up to 256 steps).  Two
// barriers per step: the update reads the fluxes of the neighbours; the
// filter reads the updated neighbours and, node by node, the filtered state
// gives the fluxes of the next step.  The thread owning the outlet node
// recomputes the two filtered values it extrapolates from.
template <typename T, int PPT>
__global__ __launch_bounds__(1024) void euler_inlet_window(T *__restrict__ state, T *__restrict__ prev, int n,
                                                           int nsteps, EulerCoef<T> c,
                                                           const double *__restrict__ theta,
                                                           const double *__restrict__ t0p) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *G = reinterpret_cast<T *>(smem_raw);
    T *X = G + EULER_GCH;
    T *Y = X + 3 * n;
    T *Fl = Y + 3 * n;
    const int bs = blockDim.x;
    T *row = state + (size_t)blockIdx.x * 3 * n;
    T *prow = prev ? prev + (size_t)blockIdx.x * 3 * n : nullptr;
    const double th0 = theta[2 * blockIdx.x], th1 = theta[2 * blockIdx.x + 1];
    const double t0 = *t0p;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = threadIdx.x + k * bs;
        if (i < n) {
            const T r = row[i], m = row[n + i], e = row[2 * n + i];
            X[i] = r;
            X[n + i] = m;
            X[2 * n + i] = e;
            euler_flux(r, m, e, c.gm1, Fl[i], Fl[n + i], Fl[2 * n + i]);
        }
    }
    for (int base = 0; base < nsteps; base += EULER_GCH) {
        const int cnt = nsteps - base < EULER_GCH ? nsteps - base : EULER_GCH;
        __syncthreads();   // fluxes written; the previous chunk's table is no longer read
        for (int q = threadIdx.x; q < cnt; q += bs) {
            const double ts = (t0 + (double)(base + q) * c.dtd) + c.dtd;
            G[q] = (T)(c.u0 * (1.0 + th0 * sin(c.omega * ts + th1))) * c.rho0;
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const int step = base + j;
            if (prow && step == nsteps - 1) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int i = threadIdx.x + k * bs;
                    if (i < n) {
                        prow[i] = X[i];
                        prow[n + i] = X[n + i];
                        prow[2 * n + i] = X[2 * n + i];
                    }
                }
            }
            // update: interior from the fluxes, inlet state, old outlet value
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = threadIdx.x + k * bs;
                if (i >= n) continue;
                if (i == 0) {
                    Y[0] = c.rho0;
                    Y[n] = G[j];
                    Y[2 * n] = c.e0;
                } else if (i < n - 1) {
#pragma unroll
                    for (int f = 0; f < 3; ++f)
                        Y[f * n + i] = X[f * n + i] + c.dt * (-(Fl[f * n + i + 1] - Fl[f * n + i - 1]) * c.inv2h);
                } else {
#pragma unroll
                    for (int f = 0; f < 3; ++f) Y[f * n + i] = X[f * n + i];
                }
            }
            __syncthreads();
            // filter, outlet extrapolation, fluxes of the new state
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = threadIdx.x + k * bs;
                if (i >= n) continue;
                T v[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const T *Yf = Y + f * n;
                    if (i == 0)
                        v[f] = Yf[0];
                    else if (i < n - 1)
                        v[f] = euler_filter_at(Yf, i, n, c.sig);
                    else
                        v[f] = T(2) * euler_filter_at(Yf, n - 2, n, c.sig) - euler_filter_at(Yf, n - 3, n, c.sig);
                    X[f * n + i] = v[f];
                }
                euler_flux(v[0], v[1], v[2], c.gm1, Fl[i], Fl[n + i], Fl[2 * n + i]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = threadIdx.x + k * bs;
        if (i < n) {
            row[i] = X[i];
            row[n + i] = X[n + i];
            row[2 * n + i] = X[2 * n + i];
        }
    }
}

// Relaxed iteration x' = x + alpha (x_prev + dt R(x) - x) of the implicit
// system (diagonal 1) at the interior; inlet node kept, outlet extrapolated
// from the iterated interior.  One thread per node, all three fields.
template <typename T>
__device__ __forceinline__ void euler_sweep_at(const T *__restrict__ x, const T *__restrict__ xp, int i, int n,
                                               T alpha, const EulerCoef<T> &c, T v[3]) {
    T fm[3], fp[3];
    euler_flux(x[i - 1], x[n + i - 1], x[2 * n + i - 1], c.gm1, fm[0], fm[1], fm[2]);
    euler_flux(x[i + 1], x[n + i + 1], x[2 * n + i + 1], c.gm1, fp[0], fp[1], fp[2]);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const T xx = x[f * n + i];
        v[f] = xx + alpha * (xp[f * n + i] + c.dt * (-(fp[f] - fm[f]) * c.inv2h) - xx);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void euler_sweep_inlet(const T *__restrict__ x, const T *__restrict__ xp,
                                                         T *__restrict__ out, int n, T alpha, EulerCoef<T> c,
                                                         const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T v[3];
    if (i == 0) {
#pragma unroll
        for (int f = 0; f < 3; ++f) v[f] = x[f * n];
    } else if (i < n - 1) {
        euler_sweep_at(x, xp, i, n, alpha, c, v);
    } else {
        T a[3], b[3];
        euler_sweep_at(x, xp, n - 2, n, alpha, c, a);
        euler_sweep_at(x, xp, n - 3, n, alpha, c, b);
#pragma unroll
        for (int f = 0; f < 3; ++f) v[f] = T(2) * a[f] - b[f];
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) out[f * n + i] = v[f];
}

size_t euler_window_lds(int n, size_t tsize) { return ((size_t)EULER_GCH + 9 * (size_t)n) * tsize; }

template <typename T>
static EulerCoef<T> euler_coef(const Plan &p, int level) {
    const int n = level == MENKF_FINE ? p.nx : p.nxc;
    const double h = p.cfg.length / n;
    const double g = p.cfg.gamma, M = p.cfg.mach;
    const double a = 1.0 / (1.0 + M), u0 = M * a, p0 = a * a / g;
    EulerCoef<T> c;
    c.dt = (T)p.cfg.dt;
    c.inv2h = (T)(1.0 / (2.0 * h));
    c.gm1 = (T)(g - 1.0);
    c.sig = (T)p.cfg.filter_sigma;
    c.rho0 = (T)1.0;
    c.e0 = (T)(p0 / (g - 1.0) + 0.5 * u0 * u0);
    c.u0 = u0;
    c.omega = p.cfg.omega;
    c.dtd = p.cfg.dt;
    return c;
}

template <typename T, int PPT>
static hipError_t launch_euler(T *state, T *prev, int n, int nb, int nsteps, EulerCoef<T> c, const double *theta,
                               const double *t0, int bs, hipStream_t s) {
    const size_t lds = euler_window_lds(n, sizeof(T));
    auto kern = euler_inlet_window<T, PPT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, s, state, prev, n, nsteps, c, theta, t0);
    return hipGetLastError();
}

template <typename T>
static hipError_t euler_forecast_t(const Plan &p, int level, T *state, int nb, int nsteps, T *prev,
                                   const double *theta, const double *t0, hipStream_t s) {
    const int n = level == MENKF_FINE ? p.nx : p.nxc;
    const EulerCoef<T> c = euler_coef<T>(p, level);
    int bs = 64;
    while (bs < 1024 && bs < n) bs *= 2;
    const int ppt = (n + bs - 1) / bs;
    if (ppt <= 1) return launch_euler<T, 1>(state, prev, n, nb, nsteps, c, theta, t0, bs, s);
    if (ppt <= 2) return launch_euler<T, 2>(state, prev, n, nb, nsteps, c, theta, t0, bs, s);
    if (ppt <= 4) return launch_euler<T, 4>(state, prev, n, nb, nsteps, c, theta, t0, bs, s);
    return hipErrorInvalidValue;   // rows this long are rejected when the context is created
}

hipError_t launch_euler_forecast(const Plan &p, int level, void *state, int nb, int nsteps, void *prev,
                                 const double *theta, const double *t0, hipStream_t s) {
    if (p.cfg.precision == MENKF_F64)
        return euler_forecast_t<double>(p, level, (double *)state, nb, nsteps, (double *)prev, theta, t0, s);
    return euler_forecast_t<float>(p, level, (float *)state, nb, nsteps, (float *)prev, theta, t0, s);
}

hipError_t launch_euler_sweep(const Plan &p, const void *x, const void *xp, void *out, double alpha,
                              const int32_t *info, hipStream_t s) {
    const int blocks = (p.nx + 255) / 256;
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(euler_sweep_inlet<double>, dim3(blocks), dim3(256), 0, s, (const double *)x,
                           (const double *)xp, (double *)out, p.nx, alpha, euler_coef<double>(p, MENKF_FINE), info);
    else
        hipLaunchKernelGGL(euler_sweep_inlet<float>, dim3(blocks), dim3(256), 0, s, (const float *)x,
                           (const float *)xp, (float *)out, p.nx, (float)alpha, euler_coef<float>(p, MENKF_FINE),
                           info);
    return hipGetLastError();
}

}  // namespace menkf
