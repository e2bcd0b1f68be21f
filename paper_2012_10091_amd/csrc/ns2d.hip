// 2D compressible Navier-Stokes forecast (Sec. 6, mass / momentum / energy
// equations) in conservative variables q = (rho, rho u, rho v, E) on a
// periodic box, fourth-order centred differences, classical RK4.
//
// Spatial operator F(q) (non-dimensional, rho0 = U0 = T0 = 1):
//   p = (gamma-1)(E - (m u + n v)/2), T = gamma Ma^2 p / rho, mu = 1/Re,
//   kappa = mu c_p / Pr, c_p = 1/((gamma-1) Ma^2), Stokes stress.
//   F_rho = -(D1x m + D1y n)
//   F_m   = -(D1x(m u + p) + D1y(m v)) + mu (4/3 D2x u + D2y u + 1/3 D1y(D1x v))
//   F_n   = -(D1x(n u) + D1y(n v + p)) + mu (D2x v + 4/3 D2y v + 1/3 D1x(D1y u))
//   F_E   = -(D1x((E+p)u) + D1y((E+p)v)) + D1x(txx u + txy v) + D1y(txy u + tyy v)
//           + kappa (D2x T + D2y T)
//   D1 f = (f[-2] - 8 f[-1] + 8 f[1] - f[2]) / 12h,
//   D2 f = (-f[-2] + 16 f[-1] - 30 f[0] + 16 f[1] - f[2]) / 12h^2,
//   txx = mu(4/3 u_x - 2/3 v_y), tyy = mu(4/3 v_y - 2/3 u_x), txy = mu(u_y + v_x).
//
// The arithmetic of one grid point is written once, in three point
// functions with every fused multiply-add explicit (FP contraction is off
// in this file), and shared by both kernel shapes, so that any schedule
// gives bitwise the same forecast:
//   ns_prim   from (rho, m, n, E): u, v, p, T, the nodal fluxes m u + p,
//             n u, m v, n v + p and E + p
//   ns_p2     from u, v at the 4 neighbours in x and in y: u_y, v_x and
//             the energy fluxes tau.u - (E+p)(u, v) (by linearity one
//             difference operator per direction covers the convective and
//             the viscous-work flux of E)
//   ns_p3     from the neighbours' fluxes, primitives and phase-2 values:
//             F(q); the difference coefficients (1/12h, mu/12h^2, ...) are
//             folded into the combining multiply-adds.
// Kernel shapes (one launch per RK stage, all members of a level in one grid):
//   ns_stage  a workgroup owns a TX x TY tile of one member; phase 1 on the
//             tile + halo 4 (u, v) / halo 2 (m, n, p, T), phase 2 on the
//             tile + halo 2, phase 3 on the tile, each staged in LDS;
//   ns_march  a workgroup owns 16 whole periodic rows of one member (rows
//             of 64 to 256 points, one thread per column) and marches down
//             them: phase 1 of row a, phase 2 of row a - 2 and phase 3 of
//             row a - 4 in one step, the y-neighbours in registers, the
//             x-neighbours in LDS rings of 5 and 3 rows, one barrier per
//             step; no x halo, a y halo of 8 rows per 16.
// The stage epilogue fuses the classical RK4 combination
//   q' = q + dt/6 (k1 + 2 k2 + 2 k3 + k4)
// with the partial sum carried where it costs no extra pass: dt/6 k1 and
// dt/3 k3 are recovered as (s1 - q)/3 and (s3 - q)/3 from the stage states
// that are read anyway, so a step moves 13 state passes instead of 16:
//   stage 1: s1 = q + dt/2 k1                              (+ x_{k-1} copy)
//   stage 2: acc = q + (s1 - q)/3 + dt/3 k2,  s2 = q + dt/2 k2
//   stage 3: s3 = q + dt k3
//   stage 4: q = acc + (s3 - q)/3 + dt/6 k4
//   sweep  : x' = x + (alpha/D)(x_prev + dt F(x) - x)     (relaxed Jacobi)
//   resid  : r = x_prev + dt F(x) - x                      (implicit-Euler residual)
#include "common.hpp"

#pragma clang fp contract(off)

namespace menkf {

template <typename T>
struct NSCoef {
    T gm1, mhgm1, tfac, epfac, half;   // gamma-1, -(gamma-1)/2, gamma Ma^2, gamma/(gamma-1), 1/2
    T ix, iy, nix, niy;                // 1/12h and -1/12h per direction
    T mu, mu2, mm23;                   // mu, 2 mu, -2/3 mu
    T vxx43, vyy, vy13;                // mu 4/3 /12hx^2, mu /12hy^2, mu/3 /12hy  (rho u equation)
    T vxx, vyy43, vx13;                // mu /12hx^2, mu 4/3 /12hy^2, mu/3 /12hx  (rho v equation)
    T kxx, kyy;                        // kappa /12h^2 per direction
    T dt, hdt, dt3, dt6, third;        // dt, dt/2, dt/3, dt/6, 1/3
    T w;                               // alpha / D for the sweep
};

enum { ST1 = 1, ST2 = 2, ST3 = 3, ST4 = 4, SWEEP = 5, RESID = 6 };

// 1/rho: the hardware reciprocal in FP32 (within 1 ulp), exact division in FP64.
__device__ __forceinline__ float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Per-point records of the LDS tiles: the values a stencil reads at one
// neighbour sit together, so each neighbour costs one wide LDS read at an
// immediate offset from a single base.
template <typename T>
struct alignas(2 * sizeof(T)) NSuv {
    T u, v;
};
template <typename T>
struct alignas(4 * sizeof(T)) NSmnpt {
    T m, n, p, tt;   // momenta, pressure, temperature
};
template <typename T>
struct alignas(2 * sizeof(T)) NSgd {
    T g, d;   // energy flux g and the cross derivative d differenced along the same direction
};
template <typename T>
struct alignas(4 * sizeof(T)) NSrx {
    T m, f1, f2, tt;   // what phase 3 differences along x: m, m u + p, n u, T
};

// ----------------------------------------------------------------- point math
template <typename T>
struct NSPrim {
    T u, v, p, tt, f1, f2, mv, nvp, ep;
};

template <typename T>
__device__ __forceinline__ T ns_rho_u2(T m, T n, T u, T v) {
    return fmad(m, u, n * v);   // rho |u|^2 = m u + n v
}

template <typename T>
__device__ __forceinline__ T ns_ep(T p, T s, const NSCoef<T> &c) {
    return fmad(c.epfac, p, c.half * s);   // E + p = gamma/(gamma-1) p + rho |u|^2 / 2
}

template <typename T>
__device__ __forceinline__ NSPrim<T> ns_prim(T rho, T m, T n, T E, const NSCoef<T> &c) {
    NSPrim<T> r;
    const T ir = recip(rho);
    r.u = m * ir;
    r.v = n * ir;
    const T s = ns_rho_u2(m, n, r.u, r.v);
    r.p = fmad(c.mhgm1, s, c.gm1 * E);
    r.tt = (c.tfac * r.p) * ir;
    r.f1 = fmad(m, r.u, r.p);
    r.f2 = n * r.u;
    r.mv = m * r.v;
    r.nvp = fmad(n, r.v, r.p);
    r.ep = ns_ep(r.p, s, c);
    return r;
}

// 12 h D1 f and 12 h^2 D2 f from the neighbours in the order -2, -1, +1, +2
template <typename T>
__device__ __forceinline__ T s1(const T f[4]) {
    return fmad(T(8), f[2] - f[1], f[0] - f[3]);
}
template <typename T>
__device__ __forceinline__ T s2(const T f[4], T f0) {
    return fmad(T(16), f[1] + f[2], fmad(T(-30), f0, -(f[0] + f[3])));
}

template <typename T>
struct NSP2 {
    T gx, gy, uy, vx;
};

// Phase 2 at one point: u, v of the x- and y-neighbours, u, v and E + p here.
template <typename T>
__device__ __forceinline__ NSP2<T> ns_p2(const T xu[4], const T xv[4], const T yu[4], const T yv[4], T u, T v,
                                         T ep, const NSCoef<T> &c) {
    const T ux = s1(xu) * c.ix, vx = s1(xv) * c.ix;
    const T uy = s1(yu) * c.iy, vy = s1(yv) * c.iy;
    const T dv = c.mm23 * (ux + vy);
    const T txx = fmad(c.mu2, ux, dv);
    const T tyy = fmad(c.mu2, vy, dv);
    const T txy = c.mu * (uy + vx);
    NSP2<T> r;
    r.gx = fmad(txx - ep, u, txy * v);   // txx u + txy v - (E+p) u
    r.gy = fmad(tyy - ep, v, txy * u);   // txy u + tyy v - (E+p) v
    r.uy = uy;
    r.vx = vx;
    return r;
}

// Phase 3 at one point: F(q) from the neighbours along x (m, m u + p, n u,
// g_x, u_y, T, u, v) and along y (n, m v, n v + p, g_y, v_x, T, u, v) and
// u, v, T here.
template <typename T>
__device__ __forceinline__ void ns_p3(const T xm[4], const T xf1[4], const T xf2[4], const T xg[4], const T xuy[4],
                                      const T xT[4], const T xu[4], const T xv[4], const T yn[4], const T ymv[4],
                                      const T ynvp[4], const T yg[4], const T yvx[4], const T yT[4], const T yu[4],
                                      const T yv[4], T u0, T v0, T T0, const NSCoef<T> &c, T k[4]) {
    k[0] = fmad(c.nix, s1(xm), c.niy * s1(yn));
    k[1] = fmad(c.nix, s1(xf1), fmad(c.niy, s1(ymv), fmad(c.vxx43, s2(xu, u0), fmad(c.vyy, s2(yu, u0), c.vy13 * s1(yvx)))));
    k[2] = fmad(c.nix, s1(xf2), fmad(c.niy, s1(ynvp), fmad(c.vxx, s2(xv, v0), fmad(c.vyy43, s2(yv, v0), c.vx13 * s1(xuy)))));
    k[3] = fmad(c.ix, s1(xg), fmad(c.iy, s1(yg), fmad(c.kxx, s2(xT, T0), c.kyy * s2(yT, T0))));
}

// The stage epilogue of one field at one point: a0, a1, a2 as the kernel
// prefetched them (ST1: q; ST2: s1, q; ST3: q; ST4: acc, q, s3; SWEEP and
// RESID: x, x_prev).
template <typename T, int MODE>
__device__ __forceinline__ void ns_epilogue(T k, T a0, T a1, T a2, const NSCoef<T> &c, T &o1, T &o2) {
    if (MODE == ST1) {
        o1 = fmad(c.hdt, k, a0);                                    // s1
    } else if (MODE == ST2) {
        o1 = fmad(c.dt3, k, fmad(c.third, a0 - a1, a1));           // acc
        o2 = fmad(c.hdt, k, a1);                                    // s2
    } else if (MODE == ST3) {
        o1 = fmad(c.dt, k, a0);                                     // s3
    } else if (MODE == ST4) {
        o1 = fmad(c.dt6, k, fmad(c.third, a2 - a1, a0));           // q'
    } else if (MODE == SWEEP) {
        o1 = fmad(c.w, fmad(c.dt, k, a1) - a0, a0);
    } else {
        o1 = fmad(c.dt, k, a1) - a0;
    }
}

template <int MODE>
struct NSPre {
    static constexpr int N = (MODE == ST1 || MODE == ST3) ? 1 : (MODE == ST4 ? 3 : 2);
};

// Loads the epilogue operands of one point (byte offset vo in the member's
// buffers) and stores its outputs.
template <typename T, int MODE>
__device__ __forceinline__ void ns_pre_load(T pre[][4], buf_t b_in, buf_t b_q0, buf_t b_acc, int vo, int fstride) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (MODE == ST1) {
            pre[0][f] = buf_load<T>(b_in, vo, f * fstride);        // q
        } else if (MODE == ST3) {
            pre[0][f] = buf_load<T>(b_q0, vo, f * fstride);        // q
        } else if (MODE == ST4) {
            pre[0][f] = buf_load<T>(b_acc, vo, f * fstride);       // acc
            pre[1][f] = buf_load<T>(b_q0, vo, f * fstride);        // q
            pre[2][f] = buf_load<T>(b_in, vo, f * fstride);        // s3
        } else {
            pre[0][f] = buf_load<T>(b_in, vo, f * fstride);        // s1 (ST2) / x
            pre[1][f] = buf_load<T>(b_q0, vo, f * fstride);        // q (ST2) / x_prev
        }
    }
}

template <typename T, int MODE>
__device__ __forceinline__ void ns_store(const T k[4], const T pre[][4], const NSCoef<T> &c, buf_t b_acc,
                                         buf_t b_next, buf_t b_out, buf_t b_prev, bool has_prev, int vo,
                                         int fstride) {
    constexpr int NP = NSPre<MODE>::N;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int so = f * fstride;
        const T a0 = pre[0][f], a1 = pre[NP > 1 ? 1 : 0][f], a2 = pre[NP - 1][f];
        T o1 = T(0), o2 = T(0);
        ns_epilogue<T, MODE>(k[f], a0, a1, a2, c, o1, o2);
        if (MODE == ST1) {
            buf_store(o1, b_next, vo, so);
            if (has_prev) buf_store(a0, b_prev, vo, so);
        } else if (MODE == ST2) {
            buf_store(o1, b_acc, vo, so);
            buf_store(o2, b_next, vo, so);
        } else if (MODE == ST3) {
            buf_store(o1, b_next, vo, so);
        } else {
            buf_store(o1, b_out, vo, so);
        }
    }
}

// ----------------------------------------------------------------- tile kernel
template <typename T, int TX, int TY, int MODE>
__global__ __launch_bounds__(256) void ns_stage(const T *__restrict__ sin_, const T *q0,
                                                T *__restrict__ acc, T *__restrict__ snext,
                                                T *qout, T *__restrict__ prev, int nx, int ny,
                                                int tiles_x, int tiles_per_member, int total_blocks,
                                                NSCoef<T> c, const int32_t *__restrict__ info) {
    constexpr int BX = TX + 8, BY = TY + 8;   // box with halo 4
    constexpr int CX = TX + 4, CY = TY + 4;   // inner box with halo 2
    constexpr int NB = BX * BY, NC = CX * CY;
    static_assert(BX + BY <= 256, "box coordinate tables are filled by one pass of the workgroup");
    __shared__ NSuv<T> suv[NB];
    // (m, n, p, T) carries one slot past the inner box that the ring of the
    // box writes to, so that phase 1 stores without a branch
    __shared__ NSmnpt<T> smp[NC + 1];
    // differenced along x: (tau.u)_x - (E+p) u and u_y; along y:
    // (tau.u)_y - (E+p) v and v_x
    __shared__ NSgd<T> sgx[NC], sgy[NC];
    __shared__ int s_col[BX], s_row[BY];   // periodic global column / row offset of the box

    if (MODE == SWEEP && *info != 0) return;   // RESID is a diagnostic: no status gate

    const int lb = xcd_remap(blockIdx.x, total_blocks);
    const int member = lb / tiles_per_member;
    const int t = lb - member * tiles_per_member;
    const int ty0 = (t / tiles_x) * TY;
    const int tx0 = (t % tiles_x) * TX;
    // this member's 4 fields of every array as buffer resources; element
    // (f, y, x) at byte offset ((f nx ny) + y nx + x) * sizeof(T)
    const int nxy = nx * ny;
    const long long mbase = (long long)member * 4 * nxy;
    const uint32_t mbytes = 4u * (uint32_t)nxy * sizeof(T);
    const int fstride = nxy * (int)sizeof(T);   // SGPR offset between fields
    const buf_t b_in = buf_rsrc(sin_ + mbase, mbytes);
    const buf_t b_q0 = buf_rsrc(q0 ? q0 + mbase : sin_, mbytes);
    const buf_t b_acc = buf_rsrc(acc ? acc + mbase : sin_, mbytes);

    // operands of the Runge-Kutta combination at the owned points, fetched
    // first so that their latency overlaps the stencil phases (stage 4
    // updates q in place: q0 and qout are the same array, each point read
    // and then written by the same thread)
    constexpr int IT3 = (TX * TY + 255) / 256;
    constexpr int NPRE = NSPre<MODE>::N;
    T pre[IT3][NPRE][4];
#pragma unroll
    for (int k = 0; k < IT3; ++k) {
        const int i = threadIdx.x + k * 256;
        const int ty = i / TX, tx = i - ty * TX;
        const int gx = tx0 + tx, gy = ty0 + ty;
        if (i < TX * TY && gx < nx && gy < ny)
            ns_pre_load<T, MODE>(pre[k], b_in, b_q0, b_acc, (gy * nx + gx) * (int)sizeof(T), fstride);
    }

    // periodic wrap of the box coordinates, once per tile
    if (threadIdx.x < BX) s_col[threadIdx.x] = wrap(tx0 - 4 + (int)threadIdx.x, nx);
    else if (threadIdx.x < BX + BY) s_row[threadIdx.x - BX] = wrap(ty0 - 4 + (int)threadIdx.x - BX, ny) * nx;
    __syncthreads();

    // phase 1: all loads of the box are issued before any is consumed.  They
    // are unconditional (E of the outer ring is read and not used; the tail
    // of the last pass re-reads the last box point): a load under a branch
    // makes the compiler wait for it before the next pass's loads go out.
    constexpr int IT1 = (NB + 255) / 256;
    T r_rho[IT1], r_m[IT1], r_n[IT1], r_E[IT1];
    int vo1[IT1];
#pragma unroll
    for (int k = 0; k < IT1; ++k) {
        const int i = min((int)threadIdx.x + k * 256, NB - 1);
        const int by = i / BX, bx = i - by * BX;
        vo1[k] = (s_row[by] + s_col[bx]) * (int)sizeof(T);
    }
#pragma unroll
    for (int k = 0; k < IT1; ++k) {
        r_rho[k] = buf_load<T>(b_in, vo1[k], 0);
        r_m[k] = buf_load<T>(b_in, vo1[k], fstride);
        r_n[k] = buf_load<T>(b_in, vo1[k], 2 * fstride);
        r_E[k] = buf_load<T>(b_in, vo1[k], 3 * fstride);
    }
#pragma unroll
    for (int k = 0; k < IT1; ++k) {
        // the tail rewrites the last box point with the value it already has
        const int i = min((int)threadIdx.x + k * 256, NB - 1);
        const int by = i / BX, bx = i - by * BX;
        const NSPrim<T> pr = ns_prim(r_rho[k], r_m[k], r_n[k], r_E[k], c);
        suv[i] = NSuv<T>{pr.u, pr.v};
        const bool inner = bx >= 2 && bx < BX - 2 && by >= 2 && by < BY - 2;
        const int ci = inner ? (by - 2) * CX + (bx - 2) : NC;
        smp[ci] = NSmnpt<T>{r_m[k], r_n[k], pr.p, pr.tt};
    }
    __syncthreads();

    // phase 2 (compile-time trip count: no loop back-edge, so the pending
    // prefetch loads are not waited for here)
    constexpr int IT2 = (NC + 255) / 256;
#pragma unroll
    for (int k2 = 0; k2 < IT2; ++k2) {
        const int i = threadIdx.x + 256 * k2;
        if (i >= NC) break;
        const int cy = i / CX, cx = i - cy * CX;
        // the box point (cx + 2, cy + 2) is pu[2 BX + 2]; every neighbour
        // read is pu[] at a non-negative constant (an immediate LDS offset)
        const NSuv<T> *pu = suv + (cy * BX + cx);
        const NSuv<T> w0 = pu[2 * BX + 2];
        const NSuv<T> xl2 = pu[2 * BX], xl1 = pu[2 * BX + 1], xr1 = pu[2 * BX + 3], xr2 = pu[2 * BX + 4];
        const NSuv<T> yl2 = pu[2], yl1 = pu[BX + 2], yr1 = pu[3 * BX + 2], yr2 = pu[4 * BX + 2];
        const T xu[4] = {xl2.u, xl1.u, xr1.u, xr2.u}, xv[4] = {xl2.v, xl1.v, xr1.v, xr2.v};
        const T yu[4] = {yl2.u, yl1.u, yr1.u, yr2.u}, yv[4] = {yl2.v, yl1.v, yr1.v, yr2.v};
        const NSmnpt<T> a0 = smp[i];
        const T ep = ns_ep(a0.p, ns_rho_u2(a0.m, a0.n, w0.u, w0.v), c);
        const NSP2<T> r = ns_p2(xu, xv, yu, yv, w0.u, w0.v, ep, c);
        sgx[i] = NSgd<T>{r.gx, r.uy};
        sgy[i] = NSgd<T>{r.gy, r.vx};
    }
    __syncthreads();

    // phase 3
    const buf_t b_next = buf_rsrc(snext ? snext + mbase : sin_, mbytes);
    const buf_t b_out = buf_rsrc(qout ? qout + mbase : sin_, mbytes);
    const buf_t b_prev = buf_rsrc(prev ? prev + mbase : sin_, mbytes);
#pragma unroll
    for (int k3 = 0; k3 < IT3; ++k3) {
        const int i = threadIdx.x + k3 * 256;
        const int ty = i / TX, tx = i - ty * TX;
        const int gx = tx0 + tx, gy = ty0 + ty;
        if (i >= TX * TY || gx >= nx || gy >= ny) continue;
        // the tile point is inner point (tx + 2, ty + 2) = pc[2 CX + 2] and
        // box point (tx + 4, ty + 4) = pb[2 BX + 2]: every read below is at a
        // non-negative constant from these bases (an immediate LDS offset)
        const int ec = ty * CX + tx, eb = (ty + 2) * BX + tx + 2;
        const NSuv<T> *pb = suv + eb;
        const NSmnpt<T> *pc = smp + ec;
        const NSgd<T> *pgx = sgx + ec, *pgy = sgy + ec;
        constexpr int OC = 2 * CX + 2, OB = 2 * BX + 2;
        // neighbour values along x (offset k) and along y, in the order
        // -2, -1, +1, +2 of the stencils
        T xm[4], xf1[4], xf2[4], xg[4], xuy[4], xT[4], xu[4], xv[4];
        T yn[4], ymv[4], ynvp[4], yg[4], yvx[4], yT[4], yu[4], yv[4];
        constexpr int offs[4] = {-2, -1, 1, 2};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int o = offs[k];
            const NSuv<T> wx = pb[OB + o];
            const NSmnpt<T> ax = pc[OC + o];
            const NSgd<T> gx_ = pgx[OC + o];
            xm[k] = ax.m;
            xf1[k] = fmad(ax.m, wx.u, ax.p);    // the values ns_prim forms
            xf2[k] = ax.n * wx.u;
            xg[k] = gx_.g;
            xuy[k] = gx_.d;
            xT[k] = ax.tt;
            xu[k] = wx.u;
            xv[k] = wx.v;
            const NSuv<T> wy = pb[OB + o * BX];
            const NSmnpt<T> ay = pc[OC + o * CX];
            const NSgd<T> gy_ = pgy[OC + o * CX];
            yn[k] = ay.n;
            ymv[k] = ay.m * wy.v;
            ynvp[k] = fmad(ay.n, wy.v, ay.p);
            yg[k] = gy_.g;
            yvx[k] = gy_.d;
            yT[k] = ay.tt;
            yu[k] = wy.u;
            yv[k] = wy.v;
        }
        const NSuv<T> w0 = pb[OB];
        const T T0 = pc[OC].tt;
        T kk[4];
        ns_p3(xm, xf1, xf2, xg, xuy, xT, xu, xv, yn, ymv, ynvp, yg, yvx, yT, yu, yv, w0.u, w0.v, T0, c, kk);
        ns_store<T, MODE>(kk, pre[k3], c, b_acc, b_next, b_out, b_prev, prev != nullptr,
                          (gy * nx + gx) * (int)sizeof(T), fstride);
    }
}

// ----------------------------------------------------------------- row-march kernel
constexpr int MARCH_ROWS = 16;
#ifndef MARCH_AHEAD_STEPS
#define MARCH_AHEAD_STEPS 1
#endif
constexpr int MARCH_AHEAD = MARCH_AHEAD_STEPS;   // steps between a row's load and its phase 1

// W threads = W columns (a whole periodic row) of one member; the
// workgroup's R = MARCH_ROWS output rows y0 .. y0 + R - 1.  Step t (fully
// unrolled, t = 0 .. R + 7) runs phase 1 on row a = y0 - 4 + t, phase 2 on
// row a - 2 (t >= 4) and phase 3 on row a - 4 (t >= 8):
//   LDS: RX, RU of row a in slot t % 5 (x-neighbours of phases 2 and 3),
//        phase 2's (g_x, u_y) in slot t % 3 (x-neighbours of phase 3);
//   registers: each thread's column of u, v, n, m v, n v + p, T (the last
//        7 rows), E + p (3 rows) and g_y, v_x (5 rows), the y-neighbours.
// A slot is rewritten 5 (3) steps after it was written, one step after its
// last reader, and a step's reads are of slots written at least two steps
// before, so one barrier at the end of every step orders all of them.
template <typename T, int W, int MODE>
__global__ __launch_bounds__(W, 4) void ns_march(const T *__restrict__ sin_, const T *q0, T *__restrict__ acc,
                                              T *__restrict__ snext, T *qout, T *__restrict__ prev, int ny,
                                              int segs, int total_blocks, NSCoef<T> c) {
    constexpr int R = MARCH_ROWS, NIT = R + 8;
    __shared__ NSrx<T> rx[5][W];
    __shared__ NSuv<T> ru[5][W];
    __shared__ NSgd<T> rb[3][W];
    const int lb = xcd_remap(blockIdx.x, total_blocks);
    const int member = lb / segs;
    const int y0 = (lb - member * segs) * R;
    const int x = threadIdx.x;
    const int xn[4] = {x >= 2 ? x - 2 : x - 2 + W, x >= 1 ? x - 1 : x - 1 + W, x + 1 < W ? x + 1 : x + 1 - W,
                       x + 2 < W ? x + 2 : x + 2 - W};
    const int nxy = W * ny;
    const long long mbase = (long long)member * 4 * nxy;
    const uint32_t mbytes = 4u * (uint32_t)nxy * sizeof(T);
    const int fstride = nxy * (int)sizeof(T);
    const buf_t b_in = buf_rsrc(sin_ + mbase, mbytes);
    const buf_t b_q0 = buf_rsrc(q0 ? q0 + mbase : sin_, mbytes);
    const buf_t b_acc = buf_rsrc(acc ? acc + mbase : sin_, mbytes);
    const buf_t b_next = buf_rsrc(snext ? snext + mbase : sin_, mbytes);
    const buf_t b_out = buf_rsrc(qout ? qout + mbase : sin_, mbytes);
    const buf_t b_prev = buf_rsrc(prev ? prev + mbase : sin_, mbytes);
    // byte offset of (row a mod ny, column x); a in [-4, ny + 3]
    auto voff = [&](int a) {
        a = a < 0 ? a + ny : (a >= ny ? a - ny : a);
        return (a * W + x) * (int)sizeof(T);
    };
    constexpr int NPRE = NSPre<MODE>::N;
    T wu[7], wv[7], wn[7], wmv[7], wnvp[7], wt[7], wep[3], wgy[5], wvx[5];
    // phase 1's input rows, loaded MARCH_AHEAD steps before they are used
    // (slot t % MARCH_AHEAD), and the epilogue operands, by step parity
    T ld[MARCH_AHEAD][4], pre[2][NPRE][4];
#pragma unroll
    for (int k = 0; k < MARCH_AHEAD; ++k) {
        const int vo = voff(y0 - 4 + k);
#pragma unroll
        for (int f = 0; f < 4; ++f) ld[k][f] = buf_load<T>(b_in, vo, f * fstride);
    }
#pragma unroll
    for (int t = 0; t < NIT; ++t) {
        // phase 1 on row a = y0 - 4 + t; the loads of row a + MARCH_AHEAD go out first
        const T rho = ld[t % MARCH_AHEAD][0], m = ld[t % MARCH_AHEAD][1], n = ld[t % MARCH_AHEAD][2],
                E = ld[t % MARCH_AHEAD][3];
        if (t + MARCH_AHEAD < NIT) {
            const int vo = voff(y0 - 4 + t + MARCH_AHEAD);
#pragma unroll
            for (int f = 0; f < 4; ++f) ld[t % MARCH_AHEAD][f] = buf_load<T>(b_in, vo, f * fstride);
        }
        if (t >= 7 && t + 1 < NIT)   // epilogue operands of the row phase 3 handles next step
            ns_pre_load<T, MODE>(pre[(t + 1) & 1], b_in, b_q0, b_acc, voff(y0 + t - 7), fstride);
        const NSPrim<T> pr = ns_prim(rho, m, n, E, c);
        rx[t % 5][x] = NSrx<T>{m, pr.f1, pr.f2, pr.tt};
        ru[t % 5][x] = NSuv<T>{pr.u, pr.v};
        wu[t % 7] = pr.u;
        wv[t % 7] = pr.v;
        wn[t % 7] = n;
        wmv[t % 7] = pr.mv;
        wnvp[t % 7] = pr.nvp;
        wt[t % 7] = pr.tt;
        wep[t % 3] = pr.ep;
        if (t >= 4) {
            // phase 2 on row a - 2 (phase 1 of step t - 2)
            const NSuv<T> *r2 = ru[(t - 2) % 5];
            const NSuv<T> q[4] = {r2[xn[0]], r2[xn[1]], r2[xn[2]], r2[xn[3]]};
            const T xu[4] = {q[0].u, q[1].u, q[2].u, q[3].u}, xv[4] = {q[0].v, q[1].v, q[2].v, q[3].v};
            const T yu[4] = {wu[(t - 4) % 7], wu[(t - 3) % 7], wu[(t - 1) % 7], wu[t % 7]};
            const T yv[4] = {wv[(t - 4) % 7], wv[(t - 3) % 7], wv[(t - 1) % 7], wv[t % 7]};
            const NSP2<T> r = ns_p2(xu, xv, yu, yv, wu[(t - 2) % 7], wv[(t - 2) % 7], wep[(t - 2) % 3], c);
            rb[t % 3][x] = NSgd<T>{r.gx, r.uy};
            wgy[t % 5] = r.gy;
            wvx[t % 5] = r.vx;
        }
        if (t >= 8) {
            // phase 3 on row y = a - 4 (phase 1 of step t - 4, phase 2 of step t - 2)
            const NSrx<T> *r3 = rx[(t - 4) % 5];
            const NSuv<T> *u3 = ru[(t - 4) % 5];
            const NSgd<T> *b3 = rb[(t - 2) % 3];
            T xm[4], xf1[4], xf2[4], xg[4], xuy[4], xT[4], xu[4], xv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const NSrx<T> a3 = r3[xn[k]];
                const NSuv<T> w3 = u3[xn[k]];
                const NSgd<T> g3 = b3[xn[k]];
                xm[k] = a3.m;
                xf1[k] = a3.f1;
                xf2[k] = a3.f2;
                xT[k] = a3.tt;
                xu[k] = w3.u;
                xv[k] = w3.v;
                xg[k] = g3.g;
                xuy[k] = g3.d;
            }
            // rows y - 2, y - 1, y + 1, y + 2: phase 1 of steps t - 6, t - 5, t - 3, t - 2
            // and phase 2 of steps t - 4, t - 3, t - 1, t
            const T yn[4] = {wn[(t - 6) % 7], wn[(t - 5) % 7], wn[(t - 3) % 7], wn[(t - 2) % 7]};
            const T ymv[4] = {wmv[(t - 6) % 7], wmv[(t - 5) % 7], wmv[(t - 3) % 7], wmv[(t - 2) % 7]};
            const T ynvp[4] = {wnvp[(t - 6) % 7], wnvp[(t - 5) % 7], wnvp[(t - 3) % 7], wnvp[(t - 2) % 7]};
            const T yT[4] = {wt[(t - 6) % 7], wt[(t - 5) % 7], wt[(t - 3) % 7], wt[(t - 2) % 7]};
            const T yu[4] = {wu[(t - 6) % 7], wu[(t - 5) % 7], wu[(t - 3) % 7], wu[(t - 2) % 7]};
            const T yv[4] = {wv[(t - 6) % 7], wv[(t - 5) % 7], wv[(t - 3) % 7], wv[(t - 2) % 7]};
            const T yg[4] = {wgy[(t - 4) % 5], wgy[(t - 3) % 5], wgy[(t - 1) % 5], wgy[t % 5]};
            const T yvx[4] = {wvx[(t - 4) % 5], wvx[(t - 3) % 5], wvx[(t - 1) % 5], wvx[t % 5]};
            T kk[4];
            ns_p3(xm, xf1, xf2, xg, xuy, xT, xu, xv, yn, ymv, ynvp, yg, yvx, yT, yu, yv, wu[(t - 4) % 7],
                  wv[(t - 4) % 7], wt[(t - 4) % 7], c, kk);
            ns_store<T, MODE>(kk, pre[t & 1], c, b_acc, b_next, b_out, b_prev, prev != nullptr, voff(y0 + t - 8),
                              fstride);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- paired row-march kernel
// Two RK stages per launch (stages 1 and 2, then 3 and 4), so that a step
// moves 7 state passes instead of 13:
//   pair 0: in q            -> acc, s2      (s1 stays on chip)       1R 2W
//   pair 1: in s2, q, acc   -> q' (into a second array)              3R 1W
// A workgroup of W threads owns PAIR_ROWS whole periodic rows of one
// member.  The first stage of the pair (A) marches exactly as ns_march
// does; each row it finishes is at once the input row of the second
// stage (B), which marches 4 rows behind.  Step t (t = 0 .. R + 15):
//   A: phase 1 on row y0 - 8 + t, phase 2 on y0 - 10 + t, phase 3 (an
//      A output row) on y0 - 12 + t;
//   B: phase 1 on that A output row, phase 2 on y0 - 14 + t, phase 3 (an
//      output row of the launch) on y0 - 16 + t.
// Each stage keeps its own LDS rings (5, 5 and 3 rows) and register
// windows, with the same ring discipline as ns_march: one barrier per step.
// The point arithmetic and the RK combinations are those of ns_stage, so
// every schedule gives bitwise the same forecast.  Pair 1 cannot update q
// in place (its y halo reads q rows that the neighbouring workgroup
// writes): it writes q' to another array and the launcher alternates the
// two between steps.

template <typename T, int W>
struct MarchRing {
    NSrx<T> rx[5][W];
    NSuv<T> ru[5][W];
    NSgd<T> rb[3][W];
};

template <typename T>
struct MarchWin {
    T wu[7], wv[7], wn[7], wmv[7], wnvp[7], wt[7], wep[3], wgy[5], wvx[5];
};

// Step s of one stage's march (compile-time after unrolling): phase 1 on
// the row whose state (rho, m, n, E) is given, phase 2 on the row of step
// s - 2 (s >= 4) and phase 3 on the row of step s - 4 (s >= 8), whose F(q)
// is returned in k.
template <int s, typename T, int W>
__device__ __forceinline__ void march_stage_step(MarchRing<T, W> &L, MarchWin<T> &w, const int x,
                                                 const int xn[4], T rho, T m, T n, T E, const NSCoef<T> &c,
                                                 T k[4]) {
    const NSPrim<T> pr = ns_prim(rho, m, n, E, c);
    L.rx[s % 5][x] = NSrx<T>{m, pr.f1, pr.f2, pr.tt};
    L.ru[s % 5][x] = NSuv<T>{pr.u, pr.v};
    w.wu[s % 7] = pr.u;
    w.wv[s % 7] = pr.v;
    w.wn[s % 7] = n;
    w.wmv[s % 7] = pr.mv;
    w.wnvp[s % 7] = pr.nvp;
    w.wt[s % 7] = pr.tt;
    w.wep[s % 3] = pr.ep;
    if constexpr (s >= 4) {
        const NSuv<T> *r2 = L.ru[(s - 2) % 5];
        const NSuv<T> q[4] = {r2[xn[0]], r2[xn[1]], r2[xn[2]], r2[xn[3]]};
        const T xu[4] = {q[0].u, q[1].u, q[2].u, q[3].u}, xv[4] = {q[0].v, q[1].v, q[2].v, q[3].v};
        const T yu[4] = {w.wu[(s - 4) % 7], w.wu[(s - 3) % 7], w.wu[(s - 1) % 7], w.wu[s % 7]};
        const T yv[4] = {w.wv[(s - 4) % 7], w.wv[(s - 3) % 7], w.wv[(s - 1) % 7], w.wv[s % 7]};
        const NSP2<T> r = ns_p2(xu, xv, yu, yv, w.wu[(s - 2) % 7], w.wv[(s - 2) % 7], w.wep[(s - 2) % 3], c);
        L.rb[s % 3][x] = NSgd<T>{r.gx, r.uy};
        w.wgy[s % 5] = r.gy;
        w.wvx[s % 5] = r.vx;
    }
    if constexpr (s >= 8) {
        const NSrx<T> *r3 = L.rx[(s - 4) % 5];
        const NSuv<T> *u3 = L.ru[(s - 4) % 5];
        const NSgd<T> *b3 = L.rb[(s - 2) % 3];
        T xm[4], xf1[4], xf2[4], xg[4], xuy[4], xT[4], xu[4], xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const NSrx<T> a3 = r3[xn[j]];
            const NSuv<T> w3 = u3[xn[j]];
            const NSgd<T> g3 = b3[xn[j]];
            xm[j] = a3.m;
            xf1[j] = a3.f1;
            xf2[j] = a3.f2;
            xT[j] = a3.tt;
            xu[j] = w3.u;
            xv[j] = w3.v;
            xg[j] = g3.g;
            xuy[j] = g3.d;
        }
        const T yn[4] = {w.wn[(s - 6) % 7], w.wn[(s - 5) % 7], w.wn[(s - 3) % 7], w.wn[(s - 2) % 7]};
        const T ymv[4] = {w.wmv[(s - 6) % 7], w.wmv[(s - 5) % 7], w.wmv[(s - 3) % 7], w.wmv[(s - 2) % 7]};
        const T ynvp[4] = {w.wnvp[(s - 6) % 7], w.wnvp[(s - 5) % 7], w.wnvp[(s - 3) % 7], w.wnvp[(s - 2) % 7]};
        const T yT[4] = {w.wt[(s - 6) % 7], w.wt[(s - 5) % 7], w.wt[(s - 3) % 7], w.wt[(s - 2) % 7]};
        const T yu[4] = {w.wu[(s - 6) % 7], w.wu[(s - 5) % 7], w.wu[(s - 3) % 7], w.wu[(s - 2) % 7]};
        const T yv[4] = {w.wv[(s - 6) % 7], w.wv[(s - 5) % 7], w.wv[(s - 3) % 7], w.wv[(s - 2) % 7]};
        const T yg[4] = {w.wgy[(s - 4) % 5], w.wgy[(s - 3) % 5], w.wgy[(s - 1) % 5], w.wgy[s % 5]};
        const T yvx[4] = {w.wvx[(s - 4) % 5], w.wvx[(s - 3) % 5], w.wvx[(s - 1) % 5], w.wvx[s % 5]};
        ns_p3(xm, xf1, xf2, xg, xuy, xT, xu, xv, yn, ymv, ynvp, yg, yvx, yT, yu, yv, w.wu[(s - 4) % 7],
              w.wv[(s - 4) % 7], w.wt[(s - 4) % 7], c, k);
    }
}

// PAIR 0: sin_ = q; writes acc, s2out and (if prev) x_{k-1} = q at the
// owned rows.  PAIR 1: sin_ = s2, q0 = q, acc read; writes qout (!= q0).
template <typename T, int W, int PAIR>
__global__ __launch_bounds__(W, 2) void ns_march_pair(const T *__restrict__ sin_, const T *__restrict__ q0,
                                                   T *__restrict__ acc, T *__restrict__ s2out,
                                                   T *__restrict__ qout, T *__restrict__ prev, int ny, int segs,
                                                   int total_blocks, NSCoef<T> c) {
    constexpr int R = PAIR_ROWS, NIT = R + 16;
    __shared__ MarchRing<T, W> LA, LB;
    const int lb = xcd_remap(blockIdx.x, total_blocks);
    const int member = lb / segs;
    const int y0 = (lb - member * segs) * R;
    const int x = threadIdx.x;
    const int xn[4] = {x >= 2 ? x - 2 : x - 2 + W, x >= 1 ? x - 1 : x - 1 + W, x + 1 < W ? x + 1 : x + 1 - W,
                       x + 2 < W ? x + 2 : x + 2 - W};
    const int nxy = W * ny;
    const long long mbase = (long long)member * 4 * nxy;
    const uint32_t mbytes = 4u * (uint32_t)nxy * sizeof(T);
    const int fstride = nxy * (int)sizeof(T);
    const buf_t b_in = buf_rsrc(sin_ + mbase, mbytes);
    const buf_t b_q = buf_rsrc((PAIR == 0 ? sin_ : q0) + mbase, mbytes);
    const buf_t b_acc = buf_rsrc(acc + mbase, mbytes);
    const buf_t b_s2 = buf_rsrc((PAIR == 0 ? s2out : acc) + mbase, mbytes);
    const buf_t b_out = buf_rsrc((PAIR == 1 ? qout : acc) + mbase, mbytes);
    const buf_t b_prev = buf_rsrc(prev ? prev + mbase : sin_, mbytes);
    // byte offset of (row a mod ny, column x); a in [-16, ny + 15]
    auto voff = [&](int a) {
        a = a < 0 ? a + ny : (a >= ny ? a - ny : a);
        return (a * W + x) * (int)sizeof(T);
    };
    MarchWin<T> wa, wb;
    // Rings indexed by step: A's input rows (6 slots: loaded one step
    // ahead, and in pair 0 also the q of A's combination four steps after
    // its load); the q rows of A's combination (pair 1; 6 slots: loaded
    // one step ahead, read again by B's combination four steps later);
    // A's outputs (5 slots, B's combination four steps later); the
    // operand of B's combination loaded one step ahead (q in pair 0, acc
    // in pair 1).  A slot is reloaded only after its last read.
    T ld[6][4], qa[6][4], sa[5][4], pb[2][4];
#pragma unroll
    for (int f = 0; f < 4; ++f) ld[0][f] = buf_load<T>(b_in, voff(y0 - 8), f * fstride);
    static_for<0, NIT>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        const int a = y0 - 8 + t;
        // loads that go out before this step's arithmetic: A's next input
        // row; (pair 1) the q row of A's combination next step; the
        // operands of B's combination next step
        if constexpr (t + 1 < NIT) {
            const int vo = voff(a + 1);
#pragma unroll
            for (int f = 0; f < 4; ++f) ld[(t + 1) % 6][f] = buf_load<T>(b_in, vo, f * fstride);
        }
        if constexpr (PAIR == 1 && t >= 7 && t + 1 < NIT) {
            const int vo = voff(y0 - 11 + t);
#pragma unroll
            for (int f = 0; f < 4; ++f) qa[(t + 1) % 6][f] = buf_load<T>(b_q, vo, f * fstride);
        }
        if constexpr (t >= 15 && t + 1 < NIT) {
            const int vo = voff(y0 - 15 + t);
#pragma unroll
            for (int f = 0; f < 4; ++f) pb[(t + 1) & 1][f] = buf_load<T>(PAIR == 0 ? b_q : b_acc, vo, f * fstride);
        }
        if constexpr (PAIR == 0 && t >= 8 && t < R + 8) {
            if (prev != nullptr) {
                const int vo = voff(a);
#pragma unroll
                for (int f = 0; f < 4; ++f) buf_store(ld[t % 6][f], b_prev, vo, f * fstride);
            }
        }
        T kA[4], kB[4];
        march_stage_step<t>(LA, wa, x, xn, ld[t % 6][0], ld[t % 6][1], ld[t % 6][2], ld[t % 6][3], c, kA);
        if constexpr (t >= 8) {
            // A's output row y0 - 12 + t (its input was loaded for step t - 4)
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                T o1 = T(0), o2 = T(0);
                if constexpr (PAIR == 0)
                    ns_epilogue<T, ST1>(kA[f], ld[(t - 4) % 6][f], T(0), T(0), c, o1, o2);
                else
                    ns_epilogue<T, ST3>(kA[f], qa[t % 6][f], T(0), T(0), c, o1, o2);
                sa[t % 5][f] = o1;
            }
            march_stage_step<t - 8>(LB, wb, x, xn, sa[t % 5][0], sa[t % 5][1], sa[t % 5][2], sa[t % 5][3], c, kB);
        }
        if constexpr (t >= 16) {
            // B's output row y0 - 16 + t
            const int vo = voff(y0 - 16 + t);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int so = f * fstride;
                T o1 = T(0), o2 = T(0);
                if constexpr (PAIR == 0) {
                    // stage 2: a0 = s1, a1 = q
                    ns_epilogue<T, ST2>(kB[f], sa[(t - 4) % 5][f], pb[t & 1][f], T(0), c, o1, o2);
                    buf_store(o1, b_acc, vo, so);
                    buf_store(o2, b_s2, vo, so);
                } else {
                    // stage 4: a0 = acc, a1 = q, a2 = s3
                    ns_epilogue<T, ST4>(kB[f], pb[t & 1][f], qa[(t - 4) % 6][f], sa[(t - 4) % 5][f], c, o1, o2);
                    buf_store(o1, b_out, vo, so);
                }
            }
        }
        __syncthreads();
    });
}

// Plain copy of n elements (the odd step of the paired schedule ends in
// the second array).
template <typename T>
__global__ __launch_bounds__(256) void copy_state(const T *__restrict__ src, T *__restrict__ dst, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

template <typename T>
static NSCoef<T> ns_coef(const Plan &p, int level, double alpha) {
    const int nx = level == MENKF_FINE ? p.nx : p.nxc;
    const int ny = level == MENKF_FINE ? p.ny : p.nyc;
    const double hx = p.cfg.length / nx, hy = p.cfg.length / ny;
    const double g = p.cfg.gamma, ma = p.cfg.mach;
    const double mu = 1.0 / p.cfg.reynolds;
    const double cp = 1.0 / ((g - 1.0) * ma * ma);
    const double kappa = mu * cp / p.cfg.prandtl;
    const double ix = 1.0 / (12.0 * hx), iy = 1.0 / (12.0 * hy);
    const double ixx = 1.0 / (12.0 * hx * hx), iyy = 1.0 / (12.0 * hy * hy);
    NSCoef<T> c;
    c.gm1 = (T)(g - 1.0);
    c.mhgm1 = (T)(-0.5 * (g - 1.0));
    c.tfac = (T)(g * ma * ma);
    c.epfac = (T)(g / (g - 1.0));
    c.half = (T)0.5;
    c.ix = (T)ix;
    c.iy = (T)iy;
    c.nix = (T)(-ix);
    c.niy = (T)(-iy);
    c.mu = (T)mu;
    c.mu2 = (T)(2.0 * mu);
    c.mm23 = (T)(-2.0 / 3.0 * mu);
    c.vxx43 = (T)(mu * 4.0 / 3.0 * ixx);
    c.vyy = (T)(mu * iyy);
    c.vy13 = (T)(mu / 3.0 * iy);
    c.vxx = (T)(mu * ixx);
    c.vyy43 = (T)(mu * 4.0 / 3.0 * iyy);
    c.vx13 = (T)(mu / 3.0 * ix);
    c.kxx = (T)(kappa * ixx);
    c.kyy = (T)(kappa * iyy);
    c.dt = (T)p.cfg.dt;
    c.hdt = (T)(0.5 * p.cfg.dt);
    c.dt3 = (T)(p.cfg.dt / 3.0);
    c.dt6 = (T)(p.cfg.dt / 6.0);
    c.third = (T)(1.0 / 3.0);
    const double D = 1.0 + p.cfg.dt * mu * (30.0 / 12.0) * (1.0 / (hx * hx) + 1.0 / (hy * hy));
    c.w = (T)(alpha / D);
    return c;
}

// Row-march schedule: rows of W = nx points (64, 128, 192 or 256, one
// thread each) and ny a multiple of the 16 rows of a workgroup (FP32).
static bool march_shape_ok(int nx, int ny) {
    return (nx == 64 || nx == 128 || nx == 192 || nx == 256) && ny % MARCH_ROWS == 0 && ny >= MARCH_ROWS;
}

template <typename T, int W>
struct MarchLauncher {
    template <int MODE>
    static hipError_t stage(const T *s, const T *q0, T *acc, T *snext, T *qout, T *prev, int ny, int nb,
                            const NSCoef<T> &c, hipStream_t st) {
        const int segs = ny / MARCH_ROWS;
        const int total = segs * nb;
        hipLaunchKernelGGL((ns_march<T, W, MODE>), dim3(total), dim3(W), 0, st, s, q0, acc, snext, qout, prev, ny,
                           segs, total, c);
        return hipGetLastError();
    }
    static hipError_t forecast(T *state, T *s1, T *s2, T *acc, T *prev, int ny, int nb, int nsteps, int chunk,
                               const NSCoef<T> &c, hipStream_t st) {
        hipError_t e = hipSuccess;
        const long long msz = 4LL * W * ny;
        if (chunk < 1 || chunk > nb) chunk = nb;
        for (int m0 = 0; m0 < nb && e == hipSuccess; m0 += chunk) {
            const int cb = nb - m0 < chunk ? nb - m0 : chunk;
            T *q = state + m0 * msz;
            T *a = acc + m0 * msz, *t1 = s1 + m0 * msz, *t2 = s2 + m0 * msz;
            T *pchunk = prev ? prev + m0 * msz : nullptr;
            for (int step = 0; step < nsteps && e == hipSuccess; ++step) {
                T *pv = step == nsteps - 1 ? pchunk : nullptr;
                e = stage<ST1>(q, nullptr, nullptr, t1, nullptr, pv, ny, cb, c, st);
                if (e == hipSuccess) e = stage<ST2>(t1, q, a, t2, nullptr, nullptr, ny, cb, c, st);
                if (e == hipSuccess) e = stage<ST3>(t2, q, nullptr, t1, nullptr, nullptr, ny, cb, c, st);
                if (e == hipSuccess) e = stage<ST4>(t1, q, a, nullptr, q, nullptr, ny, cb, c, st);
            }
        }
        return e;
    }
};

// Paired row-march schedule: rows of W = nx points (64 to 256) and ny a
// multiple of the 32 rows of a workgroup (FP32).
static bool pair_shape_ok(int nx, int ny) {
    return (nx == 64 || nx == 128 || nx == 192 || nx == 256) && ny % PAIR_ROWS == 0 && ny >= PAIR_ROWS;
}

template <typename T, int W>
struct PairLauncher {
    template <int PAIR>
    static hipError_t pair(const T *s, const T *q0, T *acc, T *s2out, T *qout, T *prev, int ny, int nb,
                           const NSCoef<T> &c, hipStream_t st) {
        const int segs = ny / PAIR_ROWS;
        const int total = segs * nb;
        hipLaunchKernelGGL((ns_march_pair<T, W, PAIR>), dim3(total), dim3(W), 0, st, s, q0, acc, s2out, qout, prev,
                           ny, segs, total, c);
        return hipGetLastError();
    }
    // q alternates between the state and the s1 array (not needed by this
    // schedule) step by step; an odd step count ends with one copy back.
    static hipError_t forecast(T *state, T *s1, T *s2, T *acc, T *prev, int ny, int nb, int nsteps, int chunk,
                               const NSCoef<T> &c, hipStream_t st) {
        hipError_t e = hipSuccess;
        const long long msz = 4LL * W * ny;
        if (chunk < 1 || chunk > nb) chunk = nb;
        for (int m0 = 0; m0 < nb && e == hipSuccess; m0 += chunk) {
            const int cb = nb - m0 < chunk ? nb - m0 : chunk;
            T *const home = state + m0 * msz;
            T *q = home, *alt = s1 + m0 * msz;
            T *a = acc + m0 * msz, *t2 = s2 + m0 * msz;
            T *pchunk = prev ? prev + m0 * msz : nullptr;
            for (int step = 0; step < nsteps && e == hipSuccess; ++step) {
                T *pv = step == nsteps - 1 ? pchunk : nullptr;
                e = pair<0>(q, nullptr, a, t2, nullptr, pv, ny, cb, c, st);
                if (e == hipSuccess) e = pair<1>(t2, q, a, nullptr, alt, nullptr, ny, cb, c, st);
                T *tmp = q;
                q = alt;
                alt = tmp;
            }
            if (e == hipSuccess && q != home) {
                const long long n = (long long)cb * msz;
                hipLaunchKernelGGL((copy_state<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, q, home, n);
                e = hipGetLastError();
            }
        }
        return e;
    }
};

template <typename T, int TX, int TY>
struct NSLauncher {
    template <int MODE>
    static hipError_t stage(const T *s, const T *q0, T *acc, T *snext, T *qout, T *prev, int nx, int ny, int nb,
                            const NSCoef<T> &c, const int32_t *info, hipStream_t st) {
        const int tiles_x = (nx + TX - 1) / TX, tiles_y = (ny + TY - 1) / TY;
        const int tpm = tiles_x * tiles_y;
        const int total = tpm * nb;
        hipLaunchKernelGGL((ns_stage<T, TX, TY, MODE>), dim3(total), dim3(256), 0, st, s, q0, acc, snext, qout,
                           prev, nx, ny, tiles_x, tpm, total, c, info);
        return hipGetLastError();
    }
    // nb states advanced member_chunk at a time through the whole window:
    // a chunk's state and RK temporaries stay resident in the last-level
    // cache across its 4 * nsteps stage launches.
    static hipError_t forecast(T *state, T *s1, T *s2, T *acc, T *prev, int nx, int ny, int nb, int nsteps,
                               int chunk, const NSCoef<T> &c, hipStream_t st) {
        hipError_t e = hipSuccess;
        const long long msz = 4LL * nx * ny;
        if (chunk < 1 || chunk > nb) chunk = nb;
        for (int m0 = 0; m0 < nb && e == hipSuccess; m0 += chunk) {
            const int cb = nb - m0 < chunk ? nb - m0 : chunk;
            T *q = state + m0 * msz;
            T *a = acc + m0 * msz, *t1 = s1 + m0 * msz, *t2 = s2 + m0 * msz;
            T *pchunk = prev ? prev + m0 * msz : nullptr;
            for (int step = 0; step < nsteps && e == hipSuccess; ++step) {
                T *pv = step == nsteps - 1 ? pchunk : nullptr;
                e = stage<ST1>(q, nullptr, nullptr, t1, nullptr, pv, nx, ny, cb, c, nullptr, st);
                if (e == hipSuccess) e = stage<ST2>(t1, q, a, t2, nullptr, nullptr, nx, ny, cb, c, nullptr, st);
                if (e == hipSuccess) e = stage<ST3>(t2, q, nullptr, t1, nullptr, nullptr, nx, ny, cb, c, nullptr, st);
                if (e == hipSuccess) e = stage<ST4>(t1, q, a, nullptr, q, nullptr, nx, ny, cb, c, nullptr, st);
            }
        }
        return e;
    }
};

// Stencil tile shapes (TX x TY points per 256-thread workgroup).  LDS per
// workgroup: (2 (TX+8)(TY+8) + 8 (TX+4)(TY+4) + 4) elements, e.g. 30.7 KB
// for 32 x 16 in FP32 (five workgroups per compute unit).  The first entry
// of each list is the default.
// The last FP32 entries are the row-march schedules (whole rows of 64 to
// 256 points): 0 x 16, one RK stage per launch and 16 rows per workgroup;
// 0 x 32, two stages per launch and 32 rows per workgroup.  On other grids
// they run the default tile.
static const int kTilesF32[][2] = {{32, 16}, {64, 8}, {32, 8}, {16, 16}, {64, 4}, {0, MARCH_ROWS}, {0, PAIR_ROWS}};
static const int kTilesF64[][2] = {{32, 8}, {16, 8}, {16, 16}, {64, 4}};

int ns_tile_count(int precision) {
    return precision == MENKF_F64 ? (int)(sizeof(kTilesF64) / sizeof(kTilesF64[0]))
                                  : (int)(sizeof(kTilesF32) / sizeof(kTilesF32[0]));
}

void ns_tile_shape(int precision, int i, int *tx, int *ty) {
    const int(*tab)[2] = precision == MENKF_F64 ? kTilesF64 : kTilesF32;
    *tx = tab[i][0];
    *ty = tab[i][1];
}

bool ns_march_applies(const Plan &p, int level, int rows) {
    const int nx = level == MENKF_FINE ? p.nx : p.nxc, ny = level == MENKF_FINE ? p.ny : p.nyc;
    if (p.dim != 2 || p.cfg.precision != MENKF_F32) return false;
    return rows == PAIR_ROWS ? pair_shape_ok(nx, ny) : rows == MARCH_ROWS && march_shape_ok(nx, ny);
}

int ns_tile_index(int precision, int tx, int ty) {
    if (tx == 0 && ty == 0) return 0;
    for (int i = 0; i < ns_tile_count(precision); ++i) {
        int a, b;
        ns_tile_shape(precision, i, &a, &b);
        if (a == tx && b == ty) return i;
    }
    return -1;
}

// Calls f.template run<TX, TY>() for the tile with index ti of the list of
// the functor's precision.
template <typename Fn>
static hipError_t with_tile(int ti, const Fn &f) {
    if constexpr (sizeof(typename Fn::T) == 8) {
        switch (ti) {
        case 1: return f.template run<16, 8>();
        case 2: return f.template run<16, 16>();
        case 3: return f.template run<64, 4>();
        default: return f.template run<32, 8>();
        }
    } else {
        switch (ti) {
        case 1: return f.template run<64, 8>();
        case 2: return f.template run<32, 8>();
        case 3: return f.template run<16, 16>();
        case 4: return f.template run<64, 4>();
        case 5: return f.run_march();
        case 6: return f.run_march_pair();
        default: return f.template run<32, 16>();
        }
    }
}

template <typename TT>
struct NSForecastFn {
    using T = TT;
    T *state, *s1, *s2, *acc, *prev;
    int nx, ny, nb, nsteps, chunk;
    NSCoef<T> c;
    hipStream_t s;
    template <int TX, int TY>
    hipError_t run() const {
        return NSLauncher<T, TX, TY>::forecast(state, s1, s2, acc, prev, nx, ny, nb, nsteps, chunk, c, s);
    }
    hipError_t run_march() const {
        if (sizeof(T) == 4 && march_shape_ok(nx, ny)) {
            switch (nx) {
            case 64: return MarchLauncher<T, 64>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            case 128: return MarchLauncher<T, 128>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            case 192: return MarchLauncher<T, 192>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            default: return MarchLauncher<T, 256>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            }
        }
        return run<32, 16>();
    }
    hipError_t run_march_pair() const {
        if (sizeof(T) == 4 && pair_shape_ok(nx, ny)) {
            switch (nx) {
            case 64: return PairLauncher<T, 64>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            case 128: return PairLauncher<T, 128>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            case 192: return PairLauncher<T, 192>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            default: return PairLauncher<T, 256>::forecast(state, s1, s2, acc, prev, ny, nb, nsteps, chunk, c, s);
            }
        }
        return run<32, 16>();
    }
};

template <typename TT, int MODE>
struct NSSingleFn {
    using T = TT;
    const T *x, *xp;
    T *out;
    int nx, ny;
    NSCoef<T> c;
    const int32_t *info;
    hipStream_t s;
    template <int TX, int TY>
    hipError_t run() const {
        return NSLauncher<T, TX, TY>::template stage<MODE>(x, xp, nullptr, nullptr, out, nullptr, nx, ny, 1, c, info, s);
    }
    hipError_t run_march() const { return run<32, 16>(); }   // sweeps and residuals use the tile kernel
    hipError_t run_march_pair() const { return run<32, 16>(); }
};

static int sched_tile(const Plan &p, int level) {
    const menkf_schedule &sc = p.sched[level == MENKF_FINE ? 0 : 1];
    const int ti = ns_tile_index(p.cfg.precision, sc.tile_x, sc.tile_y);
    return ti < 0 ? 0 : ti;
}

template <typename T>
static hipError_t ns_forecast_t(const Plan &p, int level, T *state, int nb, int nsteps, T *prev, void *ws,
                                hipStream_t s) {
    char *w = (char *)ws;
    const bool fine = level == MENKF_FINE;
    NSForecastFn<T> f;
    f.state = state;
    f.s1 = (T *)(w + (fine ? p.off_f1 : p.off_c1));
    f.s2 = (T *)(w + (fine ? p.off_f2 : p.off_c2));
    f.acc = (T *)(w + (fine ? p.off_facc : p.off_cacc));
    f.prev = prev;
    f.nx = fine ? p.nx : p.nxc;
    f.ny = fine ? p.ny : p.nyc;
    f.nb = nb;
    f.nsteps = nsteps;
    f.chunk = p.sched[fine ? 0 : 1].member_chunk;
    f.c = ns_coef<T>(p, level, 0.0);
    f.s = s;
    return with_tile(sched_tile(p, level), f);
}

hipError_t launch_ns_forecast(const Plan &p, int level, void *state, int nb, int nsteps, void *prev, void *ws,
                              hipStream_t s) {
    if (p.cfg.precision == MENKF_F64)
        return ns_forecast_t<double>(p, level, (double *)state, nb, nsteps, (double *)prev, ws, s);
    return ns_forecast_t<float>(p, level, (float *)state, nb, nsteps, (float *)prev, ws, s);
}

template <typename T>
static hipError_t ns_sweep_t(const Plan &p, const T *x, const T *xp, T *out, double alpha, const int32_t *info,
                             hipStream_t s) {
    NSSingleFn<T, SWEEP> f{x, xp, out, p.nx, p.ny, ns_coef<T>(p, MENKF_FINE, alpha), info, s};
    return with_tile(sched_tile(p, MENKF_FINE), f);
}

template <typename T>
static hipError_t ns_resid_t(const Plan &p, const T *x, const T *xp, T *out, hipStream_t s) {
    NSSingleFn<T, RESID> f{x, xp, out, p.nx, p.ny, ns_coef<T>(p, MENKF_FINE, 0.0), nullptr, s};
    return with_tile(sched_tile(p, MENKF_FINE), f);
}

hipError_t launch_ns_resid(const Plan &p, const void *x, const void *xp, void *out, hipStream_t s) {
    if (p.cfg.precision == MENKF_F64) return ns_resid_t<double>(p, (const double *)x, (const double *)xp, (double *)out, s);
    return ns_resid_t<float>(p, (const float *)x, (const float *)xp, (float *)out, s);
}

hipError_t launch_ns_sweep(const Plan &p, const void *x, const void *xp, void *out, double alpha,
                           const int32_t *info, hipStream_t s) {
    if (p.cfg.precision == MENKF_F64)
        return ns_sweep_t<double>(p, (const double *)x, (const double *)xp, (double *)out, alpha, info, s);
    return ns_sweep_t<float>(p, (const float *)x, (const float *)xp, (float *)out, alpha, info, s);
}

}  // namespace menkf
