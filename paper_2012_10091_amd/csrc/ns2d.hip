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
// Kernel structure (one launch per RK stage, all members of a level in one
// grid): a workgroup owns a TX x TY tile of one member and stages, in LDS,
//   phase 1: u, v on the tile + halo 4; m, n, p, T on the tile + halo 2
//   phase 2: u_y, v_x and the energy fluxes tau.u - (E+p)(u, v) on the tile
//            + halo 2 (by linearity one difference operator per direction
//            covers the convective and the viscous-work flux of E)
//   phase 3: F(q) at the tile points, then the stage epilogue
// The epilogue fuses the classical RK4 combination
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

namespace menkf {

template <typename T>
struct NSCoef {
    T i12hx, i12hy, i12hx2, i12hy2;
    T gm1, tfac, mu, kappa;
    T epfac;  // gamma / (gamma - 1): E + p = epfac p + (m u + n v) / 2
    T dt, w;  // w = alpha / D for the sweep
};

enum { ST1 = 1, ST2 = 2, ST3 = 3, ST4 = 4, SWEEP = 5, RESID = 6 };

// 1/rho: the hardware reciprocal in FP32 (within 1 ulp), exact division in FP64.
__device__ __forceinline__ float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }

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
    constexpr int NPRE = (MODE == ST1 || MODE == ST3) ? 1 : (MODE == ST4 ? 3 : 2);
    T pre[IT3][NPRE][4];
#pragma unroll
    for (int k = 0; k < IT3; ++k) {
        const int i = threadIdx.x + k * 256;
        const int ty = i / TX, tx = i - ty * TX;
        const int gx = tx0 + tx, gy = ty0 + ty;
        if (i < TX * TY && gx < nx && gy < ny) {
            const int vo = (gy * nx + gx) * (int)sizeof(T);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (MODE == ST1) {
                    pre[k][0][f] = buf_load<T>(b_in, vo, f * fstride);      // q
                } else if (MODE == ST3) {
                    pre[k][0][f] = buf_load<T>(b_q0, vo, f * fstride);      // q
                } else if (MODE == ST4) {
                    pre[k][0][f] = buf_load<T>(b_acc, vo, f * fstride);     // acc
                    pre[k][1][f] = buf_load<T>(b_q0, vo, f * fstride);      // q
                    pre[k][NPRE - 1][f] = buf_load<T>(b_in, vo, f * fstride);   // s3
                } else if (MODE == ST2) {
                    pre[k][0][f] = buf_load<T>(b_in, vo, f * fstride);      // s1
                    pre[k][NPRE - 1][f] = buf_load<T>(b_q0, vo, f * fstride);   // q
                } else {
                    pre[k][0][f] = buf_load<T>(b_in, vo, f * fstride);
                    pre[k][NPRE - 1][f] = buf_load<T>(b_q0, vo, f * fstride);
                }
            }
        }
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
        const T rho = r_rho[k], m = r_m[k], n = r_n[k], E = r_E[k];
        const T ir = recip(rho);
        const T u = m * ir, v = n * ir;
        suv[i] = NSuv<T>{u, v};
        const bool inner = bx >= 2 && bx < BX - 2 && by >= 2 && by < BY - 2;
        const int ci = inner ? (by - 2) * CX + (bx - 2) : NC;
        const T p = c.gm1 * (E - T(0.5) * (m * u + n * v));
        smp[ci] = NSmnpt<T>{m, n, p, c.tfac * p * ir};
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
        const T ux = (xl2.u - T(8) * xl1.u + T(8) * xr1.u - xr2.u) * c.i12hx;
        const T vx = (xl2.v - T(8) * xl1.v + T(8) * xr1.v - xr2.v) * c.i12hx;
        const T uy = (yl2.u - T(8) * yl1.u + T(8) * yr1.u - yr2.u) * c.i12hy;
        const T vy = (yl2.v - T(8) * yl1.v + T(8) * yr1.v - yr2.v) * c.i12hy;
        const T div = ux + vy;
        const T txx = c.mu * (T(2) * ux - T(2.0 / 3.0) * div);
        const T tyy = c.mu * (T(2) * vy - T(2.0 / 3.0) * div);
        const T txy = c.mu * (uy + vx);
        const T u = w0.u, v = w0.v;
        const NSmnpt<T> a0 = smp[i];
        const T ep = c.epfac * a0.p + T(0.5) * (a0.m * u + a0.n * v);   // E + p from the state
        // the energy equation's convective and viscous-work fluxes share one
        // difference operator per direction
        sgx[i] = NSgd<T>{(txx * u + txy * v) - ep * u, uy};
        sgy[i] = NSgd<T>{(txy * u + tyy * v) - ep * v, vx};
    }
    __syncthreads();

    // phase 3
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
        T xm[4], xfm[4], xfn[4], xg[4], xuy[4], xT[4], xu[4], xv[4];
        T yn[4], yfm[4], yfn[4], yg[4], yvx[4], yT[4], yu[4], yv[4];
        constexpr int offs[4] = {-2, -1, 1, 2};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int o = offs[k];
            const NSuv<T> wx = pb[OB + o];
            const NSmnpt<T> ax = pc[OC + o];
            const NSgd<T> gx_ = pgx[OC + o];
            xm[k] = ax.m;
            xfm[k] = ax.m * wx.u + ax.p;
            xfn[k] = ax.n * wx.u;
            xg[k] = gx_.g;
            xuy[k] = gx_.d;
            xT[k] = ax.tt;
            xu[k] = wx.u;
            xv[k] = wx.v;
            const NSuv<T> wy = pb[OB + o * BX];
            const NSmnpt<T> ay = pc[OC + o * CX];
            const NSgd<T> gy_ = pgy[OC + o * CX];
            yn[k] = ay.n;
            yfm[k] = ay.m * wy.v;
            yfn[k] = ay.n * wy.v + ay.p;
            yg[k] = gy_.g;
            yvx[k] = gy_.d;
            yT[k] = ay.tt;
            yu[k] = wy.u;
            yv[k] = wy.v;
        }
        const NSuv<T> w0 = pb[OB];
        const T T0 = pc[OC].tt;
#define DF(F, h) ((F[0] - T(8) * F[1] + T(8) * F[2] - F[3]) * h)
#define D2(F, f0, h) ((-F[0] + T(16) * F[1] - T(30) * (f0) + T(16) * F[2] - F[3]) * h)
        const T k_rho = -(DF(xm, c.i12hx) + DF(yn, c.i12hy));
        const T k_m = -(DF(xfm, c.i12hx) + DF(yfm, c.i12hy)) +
                      c.mu * (T(4.0 / 3.0) * D2(xu, w0.u, c.i12hx2) + D2(yu, w0.u, c.i12hy2) +
                              T(1.0 / 3.0) * DF(yvx, c.i12hy));
        const T k_n = -(DF(xfn, c.i12hx) + DF(yfn, c.i12hy)) +
                      c.mu * (D2(xv, w0.v, c.i12hx2) + T(4.0 / 3.0) * D2(yv, w0.v, c.i12hy2) +
                              T(1.0 / 3.0) * DF(xuy, c.i12hx));
        const T k_E = DF(xg, c.i12hx) + DF(yg, c.i12hy) + c.kappa * (D2(xT, T0, c.i12hx2) + D2(yT, T0, c.i12hy2));
#undef DF
#undef D2
        const T kk[4] = {k_rho, k_m, k_n, k_E};
        const int vo = (gy * nx + gx) * (int)sizeof(T);
        const buf_t b_next = buf_rsrc(snext ? snext + mbase : sin_, mbytes);
        const buf_t b_out = buf_rsrc(qout ? qout + mbase : sin_, mbytes);
        const buf_t b_prev = buf_rsrc(prev ? prev + mbase : sin_, mbytes);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int so = f * fstride;
            const T a0 = pre[k3][0][f], a1 = pre[k3][NPRE > 1 ? 1 : 0][f], a2 = pre[k3][NPRE - 1][f];
            if (MODE == ST1) {   // a0 = q
                buf_store(a0 + c.dt * T(0.5) * kk[f], b_next, vo, so);
                if (prev) buf_store(a0, b_prev, vo, so);
            } else if (MODE == ST2) {   // a0 = s1, a1 = q
                buf_store(a1 + (a0 - a1) * T(1.0 / 3.0) + c.dt * T(1.0 / 3.0) * kk[f], b_acc, vo, so);
                buf_store(a1 + c.dt * T(0.5) * kk[f], b_next, vo, so);
            } else if (MODE == ST3) {   // a0 = q
                buf_store(a0 + c.dt * kk[f], b_next, vo, so);
            } else if (MODE == ST4) {   // a0 = acc, a1 = q, a2 = s3
                buf_store(a0 + (a2 - a1) * T(1.0 / 3.0) + c.dt * T(1.0 / 6.0) * kk[f], b_out, vo, so);
            } else if (MODE == SWEEP) {
                buf_store(a0 + c.w * (a1 + c.dt * kk[f] - a0), b_out, vo, so);
            } else {
                buf_store(a1 + c.dt * kk[f] - a0, b_out, vo, so);
            }
        }
    }
}

template <typename T>
static NSCoef<T> ns_coef(const Plan &p, int level, double alpha) {
    const int nx = level == MENKF_FINE ? p.nx : p.nxc;
    const int ny = level == MENKF_FINE ? p.ny : p.nyc;
    const double hx = p.cfg.length / nx, hy = p.cfg.length / ny;
    const double g = p.cfg.gamma, ma = p.cfg.mach;
    const double mu = 1.0 / p.cfg.reynolds;
    const double cp = 1.0 / ((g - 1.0) * ma * ma);
    NSCoef<T> c;
    c.i12hx = (T)(1.0 / (12.0 * hx));
    c.i12hy = (T)(1.0 / (12.0 * hy));
    c.i12hx2 = (T)(1.0 / (12.0 * hx * hx));
    c.i12hy2 = (T)(1.0 / (12.0 * hy * hy));
    c.gm1 = (T)(g - 1.0);
    c.epfac = (T)(g / (g - 1.0));
    c.tfac = (T)(g * ma * ma);
    c.mu = (T)mu;
    c.kappa = (T)(mu * cp / p.cfg.prandtl);
    c.dt = (T)p.cfg.dt;
    const double D = 1.0 + p.cfg.dt * mu * (30.0 / 12.0) * (1.0 / (hx * hx) + 1.0 / (hy * hy));
    c.w = (T)(alpha / D);
    return c;
}

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
static const int kTilesF32[][2] = {{32, 16}, {64, 8}, {32, 8}, {16, 16}, {64, 4}};
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
