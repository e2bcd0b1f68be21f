// Ensemble Kalman analysis on the coarse level (Algo. 3 steps 3, 4, 7, 8;
// Algo. 1 steps 2-7) and the gain of the projected fine forecast x*
// (Algo. 4 step 5).
//
// With N members, N_y probes and normalised anomalies
//   X = [x^(i) - xbar]/sqrt(N-1),  Y = [H(x^(i)) - ybar]/sqrt(N-1)   (secant form),
// the gain is K = X Y^T S^-1 with S = Y Y^T + R (or Y Y^T + E E^T).  The
// state-space gain is never formed: with B = [D | d*],
// D_i = y^o + eps^(i) - H(x^(i)), d* = y^o - H(x*), the analysis needs only
//   Z = Y^T S^-1 B        (N x (N+1)),  x^a(i) = x^(i) + X Z[:, i],  delta^C = X Z[:, N].
//
// Z comes out of one FP64 Cholesky factorisation of the symmetric
// augmented matrix
//        [ S    B   Y ]            rows/cols 0..n-1      : S (padded to a block multiple with I)
//   A =  [ B^T  0   0 ]            rows n.. : B^T (N+1 rows) then Y^T (N rows)
//        [ Y^T  0   0 ]
// stopped after the first n columns: the trailing block is then the Schur
// complement -[B Y]^T S^-1 [B Y], whose (Y^T, B) block is -Z.  This folds
// the two triangular solves of S^-1 B into the factorisation's own panel
// and trailing updates.
//
// Precision: member states FP32; H(x) and anomalies in FP64; S = Y Y^T
// from BF16 anomalies on MFMA with FP32 accumulation, stored FP64;
// Cholesky, Z and the x* column (delta^C) in FP64; member update
// X Z[:, :N] on BF16 MFMA with FP32 accumulation.  MENKF_F64 contexts keep
// everything in FP64.
#include <utility>

#include "common.hpp"

namespace menkf {

// Observation perturbations: Philox stream word 0x5045 (common.hpp).
__device__ __forceinline__ double perturb_normal(uint64_t seed, uint64_t cycle, int i, int p) {
    return philox_normal(seed, cycle, i, p, 0x5045u);
}

__global__ void philox_test_kernel(const uint32_t *in, uint32_t *out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {in[6 * i], in[6 * i + 1], in[6 * i + 2], in[6 * i + 3]};
    philox4x32_10(c, in[6 * i + 4], in[6 * i + 5]);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}

// ----------------------------------------------------------------- observation operator
// y[s][p] for nb states (plus an optional extra state as row nb): H^F on the
// fine level, H^C = H^F o Pi_F (cubic Lagrange at the probe node) on the coarse level.
template <typename T>
__global__ __launch_bounds__(256) void obs_eval(const T *__restrict__ states, long long stride, int nb,
                                                const T *__restrict__ extra, const int32_t *__restrict__ idx,
                                                const int32_t *__restrict__ comp, int Ny, double *__restrict__ y,
                                                int ldy, int coarse, int dim, int nx, int ny, int r, int nxc,
                                                int nyc, int open, int obs_field) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int sidx = blockIdx.y;
    if (p >= Ny) return;
    const T *st = sidx < nb ? states + (long long)sidx * stride : extra;
    const int node = idx[p];
    const int cp = comp[p];
    double val;
    if (!coarse) {
        if (dim == 1) {
            val = (double)st[(long long)obs_field * nx + node];
        } else {
            const long long nf = (long long)nx * ny;
            const double rho = (double)st[node];
            const double mom = (double)st[(cp == 0 ? nf : 2 * nf) + node];
            val = mom / rho;
        }
    } else {
        const int fx = node % nx, fy = node / nx;
        const int jx = fx / r, mx = fx - jx * r;
        double wx[4];
        lagrange4<double>((double)mx / (double)r, wx);
        if (dim == 1 && open) {
            const int b0 = open_cubic<double>(fx, r, nxc, wx);
            const T *sf = st + (long long)obs_field * nxc;
            double a = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) a += wx[b] * (double)sf[b0 + b];
            val = a;
        } else if (dim == 1) {
            double a = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) a += wx[b] * (double)st[wrap(jx - 1 + b, nxc)];
            val = a;
        } else {
            const int jy = fy / r, my = fy - jy * r;
            double wy[4];
            lagrange4<double>((double)my / (double)r, wy);
            const long long nc = (long long)nxc * nyc;
            const T *rho_f = st;
            const T *mom_f = st + (cp == 0 ? nc : 2 * nc);
            double rho = 0.0, mom = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const long long row = (long long)wrap(jy - 1 + a, nyc) * nxc;
                double ra = 0.0, ma = 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const long long g = row + wrap(jx - 1 + b, nxc);
                    ra += wx[b] * (double)rho_f[g];
                    ma += wx[b] * (double)mom_f[g];
                }
                rho += wy[a] * ra;
                mom += wy[a] * ma;
            }
            val = mom / rho;
        }
    }
    y[(long long)sidx * ldy + p] = val;
}

// ----------------------------------------------------------------- anomalies and innovations
// One thread per (padded) probe p.  Writes, in FP64,
//   Yk[p][0..N) = Y_p, Yk[p][N..2N) = E_p in sample mode, zero up to kdim;
//   A[(nyp + j) ld + p] = D_pj (j < N), d*_p (j = N), Y_p,j-N-1 (N < j <= 2N).
// S and the right-hand sides are built from the very same Y values: S^-1
// amplifies any inconsistency between them by up to 1/sigma^2.
__global__ __launch_bounds__(256) void obs_pack(const double *__restrict__ yraw, int ldy, int N, int Ny, int nyp,
                                                const double *__restrict__ yobs, const double *__restrict__ eps,
                                                uint64_t seed, uint64_t cycle, const uint64_t *__restrict__ dcycle,
                                                double sigma, int sample_mode, double *__restrict__ Yk, int kdim,
                                                double *__restrict__ A, int ld, int with_xstar) {
    // 16 probes per workgroup, the members of a probe split over 16 lanes
    // (member i goes to group i % 16); the member means are reduced in a
    // fixed order through LDS.
    __shared__ double red[2][16][16];
    const int pl = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int p = blockIdx.x * 16 + pl;
    if (dcycle) cycle = *dcycle;
    const bool live = p < Ny;
    double ys = 0.0, es = 0.0;
    if (live) {
        for (int i = g; i < N; i += 16) {
            ys += yraw[(long long)i * ldy + p];
            if (sample_mode) es += eps ? eps[(long long)i * Ny + p] : sigma * perturb_normal(seed, cycle, i, p);
        }
    }
    red[0][g][pl] = ys;
    red[1][g][pl] = es;
    __syncthreads();
    double ybar = 0.0, ebar = 0.0;
#pragma unroll
    for (int gg = 0; gg < 16; ++gg) {
        ybar += red[0][gg][pl];
        ebar += red[1][gg][pl];
    }
    ybar /= (double)N;
    ebar /= (double)N;
    if (p >= nyp) return;
    double *yk = Yk + (long long)p * kdim;
    double *B = A + (long long)nyp * ld + p;
    if (!live) {   // padding probe
        for (int k = g; k < kdim; k += 16) yk[k] = 0.0;
        for (int j = g; j <= 2 * N; j += 16) B[(long long)j * ld] = 0.0;
        return;
    }
    const double scale = 1.0 / sqrt((double)(N - 1));
    const double yo = yobs[p];
    for (int i = g; i < N; i += 16) {
        const double yi = yraw[(long long)i * ldy + p];
        const double e = eps ? eps[(long long)i * Ny + p] : sigma * perturb_normal(seed, cycle, i, p);
        const double an = (yi - ybar) * scale;
        yk[i] = an;
        B[(long long)i * ld] = yo + e - yi;
        B[(long long)(N + 1 + i) * ld] = an;
        if (sample_mode) yk[N + i] = (e - ebar) * scale;
    }
    for (int k = (sample_mode ? 2 * N : N) + g; k < kdim; k += 16) yk[k] = 0.0;
    if (g == 0) B[(long long)N * ld] = with_xstar ? yo - yraw[(long long)N * ldy + p] : 0.0;
}

// Zero the trailing (Schur) block and the padding rows of the extra block,
// and reset the status word for this factorisation.
__global__ __launch_bounds__(256) void zero_extra(double *__restrict__ A, int ld, int nyp, int mext,
                                                  int32_t *__restrict__ info) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = 0;
    const int rows = ld - nyp;
    const long long tot = (long long)rows * ld;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(t / ld), c = (int)(t - (long long)a * ld);
        if (c >= nyp || a >= mext) A[(long long)(nyp + a) * ld + c] = 0.0;
    }
}

__device__ __forceinline__ void tri_index(int t, int &bi, int &bj) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    bi = i;
    bj = t - i * (i + 1) / 2;
}

// ----------------------------------------------------------------- blocked FP64 Cholesky
// Right-looking, block size 64, on the lower triangle of A (row-major,
// element (r, c) at r*ld + c, r >= c).  Step k: factor the diagonal block
// and invert its factor (one wave), panel X = A_ik L_kk^-T for every block
// row below (including the extra rows), trailing update A_ij -= L_ik L_jk^T
// for k < j <= i over the whole matrix (the extra rows accumulate the Schur
// complement).  Every kernel exits if the status word is set.
constexpr int LDP = 65;  // padded LDS row (doubles)

// 1/p for the pivot chain: the hardware reciprocal y (relative error below
// 2^-24 on gfx950) refined by the third-order step y (1 + e + e^2), e =
// 1 - p y, whose error ~e^3 is far below the rounding of the result (it
// matched the correctly rounded 1/p on every one of 4M log-uniform samples
// over 2^+-700, as did two Newton steps); three dependent FMAs after the
// reciprocal, against four for two Newton steps and about twice that for
// the correctly rounded division: the pivot reciprocal is the longest part
// of a pivot step.
__device__ __forceinline__ double pivot_recip(double p) {
    const double y = __builtin_amdgcn_rcp(p);
    const double e = fma(-p, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

// Factor the 64x64 diagonal block and invert its factor in one sweep of
// 64 pivot steps.  W is the block being reduced (columns are never rescaled
// in place) and X the rows of the inverse in unscaled form; at step j,
// with m_r = W[r][j] / W[j][j] for r > j (0 otherwise),
//   W[r][c] -= m_r W[c][j]   (c > j)        Schur update
//   X[r][c] -= m_r X[j][c]   (all c)        inverse rows (X[j][c] = 0 for c > j)
// and at the end L[r][c] = W[r][c] / d_c with d_c = sqrt(W[c][c]) at its
// step, L^-1[r][c] = X[r][c] / d_r.
// Thread t owns the 4x4 blocks (rows 4a..4a+3, columns 4b..4b+3, a = t / 16,
// b = t % 16) of W and X in registers.  Step j publishes, double-buffered in
// LDS, the column v = W[:, j] with zeros at rows <= j (so the update of
// finished columns and of column j itself is a no-op and needs no test),
// the row X[j][:] and 1/W[j][j]; every owned entry is then updated with
// m = v * (1/W[j][j]): one barrier per pivot, no per-column branches.
// The entries the next step publishes (column j + 1, row j + 1 of X, the
// pivot, whose owner computes its reciprocal) are updated and written first
// so that their latency overlaps the rest of the update.  A pivot that is
// not positive publishes -1 as its reciprocal; it is recorded and the
// sweep runs to the end (no early exit inside the pivot loop) before the
// status word is set.
// The block is read from src (row stride lds_: global A or an LDS copy) and
// the factor written to Ak (row stride ld).  256 threads; must be entered by
// the whole workgroup.
__device__ __forceinline__ void chol_diag_block(const double *src, long long lds_, double *__restrict__ Ak,
                                                long long ld, int k, double *__restrict__ Linv,
                                                int32_t *__restrict__ info) {
    // The pivot chain is the critical path of the factorisation and issues
    // little; when other kernels share its compute unit (a forecast on a
    // second stream), the highest wave priority lets it issue first.
    __builtin_amdgcn_s_setprio(3);
    __shared__ __attribute__((aligned(16))) double colbuf[2][64];
    __shared__ __attribute__((aligned(16))) double rowbuf[2][64];
    __shared__ double invbuf[2];
    __shared__ double pivbuf[64];
    const int t = threadIdx.x;
    const int a = t >> 4, b = t & 15;
    double w[4][4], x[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * a + i, c = 4 * b + q;
            w[i][q] = c <= r ? src[(long long)r * lds_ + c] : 0.0;
            x[i][q] = c == r ? 1.0 : 0.0;
        }
    // step 0's column, row and pivot
    if (b == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) colbuf[0][4 * a + i] = 4 * a + i > 0 ? w[i][0] : 0.0;
    }
    if (a == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) rowbuf[0][4 * b + q] = x[0][q];
    }
    if (t == 0) {
        const double p = w[0][0];
        pivbuf[0] = p;
        invbuf[0] = p > 0.0 ? pivot_recip(p) : -1.0;
    }
    __syncthreads();
    int bad = 0;
    for (int jb = 0; jb < 16; ++jb) {
#pragma unroll
        for (int jc = 0; jc < 4; ++jc) {
            const int j = 4 * jb + jc;
            const int buf = jc & 1;
            // every read of the step is issued before any is used
            const double inv = invbuf[buf];
            const double2 *cb = (const double2 *)colbuf[buf];
            const double2 *rb = (const double2 *)rowbuf[buf];
            const double2 cr0 = cb[2 * a], cr1 = cb[2 * a + 1];
            const double2 vc0 = cb[2 * b], vc1 = cb[2 * b + 1];
            const double2 xr0 = rb[2 * b], xr1 = rb[2 * b + 1];
            if (!(inv > 0.0) && bad == 0) bad = j + 1;
            const double m[4] = {cr0.x * inv, cr0.y * inv, cr1.x * inv, cr1.y * inv};
            const double v[4] = {vc0.x, vc0.y, vc1.x, vc1.y};
            const double xr[4] = {xr0.x, xr0.y, xr1.x, xr1.y};
            const int jc1 = (jc + 1) & 3;   // local column / row of index j + 1
            const int jb1 = (j + 1) >> 2;
#pragma unroll
            for (int i = 0; i < 4; ++i) w[i][jc1] -= m[i] * v[jc1];
#pragma unroll
            for (int q = 0; q < 4; ++q) x[jc1][q] -= m[jc1] * xr[q];
            if (j + 1 < 64) {
                if (b == jb1) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) colbuf[buf ^ 1][4 * a + i] = 4 * a + i > j + 1 ? w[i][jc1] : 0.0;
                    if (a == jb1) {
                        const double p = w[jc1][jc1];
                        pivbuf[j + 1] = p;
                        invbuf[buf ^ 1] = p > 0.0 ? pivot_recip(p) : -1.0;
                    }
                }
                if (a == jb1) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) rowbuf[buf ^ 1][4 * b + q] = x[jc1][q];
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q != jc1) w[i][q] -= m[i] * v[q];
                    if (i != jc1) x[i][q] -= m[i] * xr[q];
                }
            __syncthreads();
        }
    }
    if (bad) {
        if (t == 0) *info = k * 64 + bad;
        return;
    }
    // pivots -> d_c and 1/d_c, one division per pivot: the 32 entries of
    // each thread are then scaled by multiplications
    __shared__ double dsq[64], rdsq[64];
    if (t < 64) {
        const double d = sqrt(pivbuf[t]);
        dsq[t] = d;
        rdsq[t] = 1.0 / d;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * a + i;
        const double dr = dsq[r], rdr = rdsq[r];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * b + q;
            if (c <= r) Ak[(long long)r * ld + c] = c == r ? dr : w[i][q] * rdsq[c];
            Linv[r * 64 + c] = c <= r ? x[i][q] * rdr : 0.0;
        }
    }
}

// ---- hierarchical form of the same factorisation (64x64 block, 256 threads)
// The block is split into 4 x 4 sub-blocks of 16 x 16.  For s = 0..3:
//   F: one wave factors the diagonal sub-block, D_ss = L_ss L_ss^T, and
//      inverts L_ss: a 16-pivot sweep held in registers, no barrier
//      inside (the pivot column reaches the lanes by a row broadcast within
//      each 16-lane row, the pivot row by a lane permute);
//   P: L_is = D_is L_ss^-T for the sub-blocks below (16x16x16 on FP64 MFMA);
//   U: D_ij -= L_is L_js^T for s < j <= i (FP64 MFMA).
// Then the blocks of L^-1 below the diagonal, by distance from it:
//   (L^-1)_ij = -L_ii^-1 sum_{k=j}^{i-1} L_ik (L^-1)_kj,  (L^-1)_jj = L_jj^-1.
// The pivots are those of the unblocked sweep (the diagonal of the
// successive Schur complements); a pivot that is not positive is recorded
// and the first one reported through the status word, outputs untouched.
// In the 16-pivot sweep the block being reduced and the rows of the
// inverse are both unscaled, as in chol_diag_block; at the end
// L[r][c] = W[r][c] / sqrt(p_c) and L^-1[r][c] = X[r][c] / sqrt(p_r).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// value of lane J of the caller's 16-lane row (DPP row broadcast)
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x150 + J, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x150 + J, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// 16x16 factor and inverse of the sub-block at Ws (row stride LDP, lower
// triangle read), by one wave: L_ss over the lower triangle of Ws (zeros
// above), L_ss^-1 into Ts (16 x 16, zeros above), the pivots into piv[16].
// Returns 1 + the first non-positive pivot (0 if none); uniform.
// Lane l holds column c = l % 16 of W, rows r = 4 (l / 16) + e, and the
// inverse rows transposed: xt[e] = X[c][r].  With m_c = W[j][c] / p_j for
// c > j (0 otherwise), step j is
//   W[r][c] -= W[r][j] m_c     (every r: rows r <= j change only above the
//                               diagonal, which is never read back)
//   X[c][k] -= m_c X[j][k]     (X[j][k]: lane j of the caller's 16-lane row)
// so both updates share the one per-lane multiplier m_c and need no mask on
// the rows; the pivot column and X[j][.] arrive by row broadcasts, the
// pivot row by a lane permute.
__device__ __forceinline__ int chol16_wave(double *Ws, double *Ts, double *piv) {
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    double w[4], xt[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = 4 * q + e;
        w[e] = r >= c ? Ws[r * LDP + c] : Ws[c * LDP + r];
        xt[e] = r == c ? 1.0 : 0.0;
    }
    static_for<0, 16>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int jq = j >> 2, je = j & 3;
        const double p = readlane_d(w[je], 16 * jq + j);   // W[j][j]
        const double inv = pivot_recip(p);   // garbage after a bad pivot: the outputs are not written then
        const double rowj = __shfl(w[je], 16 * jq + c);   // W[j][c]
        const double mc = c > j ? rowj * inv : 0.0;
        double colj[4], xj[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) colj[e] = row_bcast<j>(w[e]);    // W[4 q + e][j]
#pragma unroll
        for (int e = 0; e < 4; ++e) xj[e] = row_bcast<j>(xt[e]);     // X[j][4 q + e]
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = fma(-colj[e], mc, w[e]);
#pragma unroll
        for (int e = 0; e < 4; ++e) xt[e] = fma(-mc, xj[e], xt[e]);
    });
    // the diagonal of w is the pivot sequence
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (4 * q + e == c) piv[c] = w[e];
    wave_sync();
    const double pc = piv[c];
    const unsigned long long nonpos = __ballot(l < 16 && !(pc > 0.0));
    const int bad = nonpos ? __builtin_ctzll(nonpos) + 1 : 0;
    const double rdc = 1.0 / sqrt(pc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = 4 * q + e;
        Ws[r * LDP + c] = r > c ? w[e] * rdc : (r == c ? sqrt(pc) : 0.0);
        Ts[c * 16 + r] = c >= r ? xt[e] * rdc : 0.0;   // L^-1[c][r] = X[c][r] / d_c
    }
    return bad;
}
// acc (16x16, MFMA result layout) += A B over K = 16: A at Pa (row stride
// lda), B given transposed (Bt[n][k]) at Pb (row stride ldb).  One wave.
__device__ __forceinline__ void mfma16_nt(const double *Pa, int lda, const double *Pb, int ldb, f64x4 &acc) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
        const double a = Pa[(l & 15) * lda + k0 + (l >> 4)];
        const double b = Pb[(l & 15) * ldb + k0 + (l >> 4)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
}

// acc (16x16) += A B over K = 16 with B in natural layout (B[k][n] at Pb,
// row stride ldb).  One wave.
__device__ __forceinline__ void mfma16_nn(const double *Pa, int lda, const double *Pb, int ldb, f64x4 &acc) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
        const double a = Pa[(l & 15) * lda + k0 + (l >> 4)];
        const double b = Pb[(k0 + (l >> 4)) * ldb + (l & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
}

// element e of lane l of an MFMA result: row 4 e + l / 16, column l % 16
template <typename Fn>
__device__ __forceinline__ void for_acc16(const f64x4 &acc, Fn f) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int e = 0; e < 4; ++e) f(4 * e + (l >> 4), l & 15, acc[e]);
}

// Hierarchical factorisation of the 64x64 block held in LDS at W (row
// stride LDP, lower triangle; overwritten by L), with LDS scratch of
// DIAG_SCRATCH doubles; L to Ak (row stride ld), L^-1 to Linv (64 x 64,
// zeros above).  256 threads; must be entered by the whole workgroup.
constexpr int DIAG_SCRATCH = 4 * 256 + 6 * 256 + 4 * 256 + 64 + 8;
__device__ __forceinline__ void chol_diag_hier(double *W, double *scr, double *__restrict__ Ak, long long ld, int k,
                                               double *__restrict__ Linv, int32_t *__restrict__ info,
                                               long long *stamps = nullptr) {
    int nst = 0;
    auto stamp = [&]() {
        if (stamps && threadIdx.x == 0) stamps[nst] = (long long)__builtin_amdgcn_s_memtime();
        ++nst;
    };
    stamp();
    __builtin_amdgcn_s_setprio(3);
    double *Ti = scr;                  // 4 x (16 x 16): L_ss^-1
    double *V = scr + 4 * 256;         // 6 x (16 x 16): (L^-1)_ij, i > j, block index ij_index(i, j)
    double *Tw = scr + 10 * 256;       // 4 x (16 x 16): one per wave
    double *piv = scr + 14 * 256;      // 64 pivots
    int *badw = reinterpret_cast<int *>(scr + 14 * 256 + 64);
    const int tid = threadIdx.x, wave = tid >> 6;
    auto vidx = [](int i, int j) { return (i * (i - 1)) / 2 + j; };   // (1,0)=0 (2,0)=1 (2,1)=2 (3,0)=3 ...
    if (tid == 0) *badw = 0;
    __syncthreads();
    // wave 0 carries the chain F(s) -> P(s) -> update of D_{s+1,s+1} ->
    // F(s+1); the other waves update the rest of the trailing blocks and
    // form the blocks of L^-1 beside it
    auto factor = [&](int s) {
        const int b = chol16_wave(W + 16 * s * LDP + 16 * s, Ti + 256 * s, piv + 16 * s);
        if (b && (threadIdx.x & 63) == 0 && *badw == 0) *badw = 16 * s + b;
    };
    auto update = [&](int s, int i, int j) {   // D_ij -= L_is L_js^T
        double *Dij = W + 16 * i * LDP + 16 * j;
        f64x4 acc = {};
        mfma16_nt(W + 16 * i * LDP + 16 * s, LDP, W + 16 * j * LDP + 16 * s, LDP, acc);
        double old[4];
        for_acc16(acc, [&](int r, int cc, double) { old[r >> 2] = Dij[r * LDP + cc]; });
        for_acc16(acc, [&](int r, int cc, double v) { Dij[r * LDP + cc] = old[r >> 2] - v; });
    };
    auto inverse_block = [&](int i, int j) {   // (L^-1)_ij = -L_ii^-1 sum_{k=j}^{i-1} L_ik (L^-1)_kj
        f64x4 acc = {};
        mfma16_nn(W + 16 * i * LDP + 16 * j, LDP, Ti + 256 * j, 16, acc);
        for (int kk = j + 1; kk < i; ++kk) mfma16_nn(W + 16 * i * LDP + 16 * kk, LDP, V + 256 * vidx(kk, j), 16, acc);
        double *T = Tw + 256 * wave;
        for_acc16(acc, [&](int r, int cc, double v) { T[r * 16 + cc] = v; });
        wave_sync();
        f64x4 acc2 = {};
        mfma16_nn(Ti + 256 * i, 16, T, 16, acc2);
        double *Vij = V + 256 * vidx(i, j);
        for_acc16(acc2, [&](int r, int cc, double v) { Vij[r * 16 + cc] = -v; });
    };
    if (wave == 0) factor(0);
    __syncthreads();
    stamp();
    for (int s = 0; s < 4; ++s) {
        // panels L_is = D_is L_ss^-T (waves 0 .. 2 - s); the blocks
        // (L^-1)_sj, j < s, on the waves left (they need L_ss^-1, the final
        // L_s. and the (L^-1)_kj of the earlier stages)
        if (wave < 3 - s) {
            const int i = s + 1 + wave;
            double *Dis = W + 16 * i * LDP + 16 * s;
            f64x4 acc = {};
            mfma16_nt(Dis, LDP, Ti + 256 * s, 16, acc);
            for_acc16(acc, [&](int r, int cc, double v) { Dis[r * LDP + cc] = v; });
        } else if (wave - (3 - s) < s) {
            inverse_block(s, wave - (3 - s));
        }
        __syncthreads();
        stamp();
        if (s == 3) break;
        // trailing update; wave 0 takes D_{s+1,s+1} and factors it at once
        if (wave == 0) {
            update(s, s + 1, s + 1);
            wave_sync();
            factor(s + 1);
        } else {
            const int nb = 3 - s, nt = nb * (nb + 1) / 2;
            for (int t = 1 + (wave - 1); t < nt; t += 3) {   // block t = 0 is D_{s+1,s+1}
                int bi = 0;
                while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
                const int bj = t - bi * (bi + 1) / 2;
                update(s, s + 1 + bi, s + 1 + bj);
            }
        }
        __syncthreads();
        stamp();
    }
    const int bad = *badw;
    if (bad) {
        if (tid == 0) *info = k * 64 + bad;
        return;
    }
    // outputs: L (lower) and L^-1 (zeros above the diagonal), each wave 16
    // whole rows (one 512-byte store per row and array)
    {
        const int c = tid & 63, bj = c >> 4;
        for (int rr = 0; rr < 16; ++rr) {
            const int r = 16 * wave + rr, bi = r >> 4;
            if (c <= r) Ak[(long long)r * ld + c] = W[r * LDP + c];
            double v = 0.0;
            if (bj == bi)
                v = Ti[256 * bi + (r & 15) * 16 + (c & 15)];
            else if (bj < bi)
                v = V[256 * vidx(bi, bj) + (r & 15) * 16 + (c & 15)];
            Linv[r * 64 + c] = v;
        }
    }
    stamp();
}

#ifndef CHOL_DIAG_HIER
#define CHOL_DIAG_HIER 1
#endif

__global__ __launch_bounds__(256) void chol_diag(double *__restrict__ A, int ld, int k, double *__restrict__ Linv,
                                                 int32_t *__restrict__ info) {
    if (*info != 0) return;
    double *Ak = A + (long long)(k * 64) * ld + k * 64;
#if CHOL_DIAG_HIER
    __shared__ __attribute__((aligned(16))) double Wd[64 * LDP];
    __shared__ __attribute__((aligned(16))) double scr[DIAG_SCRATCH];
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        if (c <= r) Wd[r * LDP + c] = Ak[(long long)r * ld + c];
    }
    __syncthreads();
    chol_diag_hier(Wd, scr, Ak, ld, k, Linv, info);
#else
    chol_diag_block(Ak, ld, Ak, ld, k, Linv, info);
#endif
}

// acc += P Q^T for 64-row blocks P (rows of length K at ldp) and Q, K a
// multiple of 64, staged 64 columns at a time through LDS.  FP64 MFMA
// 16x16x4; 4 waves, each a 32x32 quarter held as 2x2 16x16 accumulators.
// v_mfma_f64_16x16x4f64: lane l holds A(l % 16, l / 16), B(l / 16, l % 16);
// result element e of lane l is row 4 e + l / 16, column l % 16.
__device__ __forceinline__ void mfma_nt_64_acc(const double *__restrict__ P, long long ldp,
                                               const double *__restrict__ Q, long long ldq, int K,
                                               f64x4 (&acc)[2][2], double *Ps, double *Qs) {
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    for (int k0 = 0; k0 < K; k0 += 64) {
        // all 32 loads of this thread are issued before the first LDS store
        double pv[16], qv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int r = (tid >> 6) + 4 * j, c = tid & 63;
            pv[j] = P[r * ldp + k0 + c];
            qv[j] = Q[r * ldq + k0 + c];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int r = (tid >> 6) + 4 * j, c = tid & 63;
            Ps[r * LDP + c] = pv[j];
            Qs[r * LDP + c] = qv[j];
        }
        __syncthreads();
        for (int kk = 0; kk < 64; kk += 4) {
            const int kcol = kk + (l >> 4);
            double a[2], b[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                a[s] = Ps[(r0 + s * 16 + (l & 15)) * LDP + kcol];
                b[s] = Qs[(c0 + s * 16 + (l & 15)) * LDP + kcol];
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[u], acc[s][u], 0, 0, 0);
        }
    }
}

// The (row, col) positions of this thread's accumulator entries, in the
// order for_each_acc visits them.
template <typename Fn>
__device__ __forceinline__ void for_each_pos(Fn f) {
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) f(r0 + s * 16 + 4 * e + (l >> 4), c0 + u * 16 + (l & 15));
}

// Visit the accumulator entries: f(row, col, value) within the 64x64 block.
template <typename Fn>
__device__ __forceinline__ void for_each_acc(const f64x4 (&acc)[2][2], Fn f) {
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) f(r0 + s * 16 + 4 * e + (l >> 4), c0 + u * 16 + (l & 15), acc[s][u][e]);
}

// C (64x64, ldc) = beta*C + sgn * P Q^T with K = 64.
__device__ __forceinline__ void gemm_nt_64(const double *__restrict__ P, long long ldp, const double *__restrict__ Q,
                                           long long ldq, double *__restrict__ C, long long ldc, double beta,
                                           double sgn, double *Ps, double *Qs, bool lower_only) {
    f64x4 acc[2][2] = {};
    mfma_nt_64_acc(P, ldp, Q, ldq, 64, acc, Ps, Qs);
    if (beta != 0.0) {
        // read the 16 old values of this thread before any store
        double old[16];
        int n = 0;
        for_each_pos([&](int r, int c) { old[n++] = (lower_only && c > r) ? 0.0 : C[(long long)r * ldc + c]; });
        n = 0;
        for_each_acc(acc, [&](int r, int c, double v) {
            const double o = old[n++];
            if (lower_only && c > r) return;
            C[(long long)r * ldc + c] = beta * o + sgn * v;
        });
    } else {
        for_each_acc(acc, [&](int r, int c, double v) {
            if (lower_only && c > r) return;
            C[(long long)r * ldc + c] = sgn * v;
        });
    }
}

// S = Yk Yk^T + R on the lower 64x64 blocks (identity on the padding rows).
__global__ __launch_bounds__(256) void syrk_f64_mfma(const double *__restrict__ Yk, int kdim, int Ny, double r_diag,
                                                     double *__restrict__ A, int ld) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    int bi, bj;
    tri_index(blockIdx.x, bi, bj);
    f64x4 acc[2][2] = {};
    mfma_nt_64_acc(Yk + (long long)bi * 64 * kdim, kdim, Yk + (long long)bj * 64 * kdim, kdim, kdim, acc, smem_d,
                   smem_d + 64 * LDP);
    double *C = A + (long long)(bi * 64) * ld + bj * 64;
    for_each_acc(acc, [&](int r, int c, double v) {
        const int p = bi * 64 + r, q = bj * 64 + c;
        if (q > p) return;
        if (p == q) v += p < Ny ? r_diag : 1.0;
        C[(long long)r * ld + c] = v;
    });
}

__global__ __launch_bounds__(256) void chol_panel(double *__restrict__ A, int ld, int k, const double *__restrict__ Linv,
                                                  const int32_t *__restrict__ info) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    if (*info != 0) return;
    __builtin_amdgcn_s_setprio(3);   // on the factorisation's critical path, like the diagonal block
    const int i = k + 1 + blockIdx.x;
    double *Aik = A + (long long)(i * 64) * ld + k * 64;
    // X = A_ik Linv^T, in place (A_ik is staged in LDS before any write)
    gemm_nt_64(Aik, ld, Linv, 64, Aik, ld, 0.0, 1.0, smem_d, smem_d + 64 * LDP, false);
}

// Trailing update of step k.  Workgroup 0 owns the next diagonal block
// (k+1, k+1): when k+1 < nbs it keeps its updated block in LDS and
// factors it right away (look-ahead), overlapping the latency-bound pivot
// chain of step k+1 with the other blocks of step k.
__global__ __launch_bounds__(256) void chol_update(double *__restrict__ A, int ld, int k, int nbs,
                                                   double *__restrict__ Linv, int32_t *__restrict__ info) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    if (*info != 0) return;
    int bi, bj;
    tri_index(blockIdx.x, bi, bj);
    const int i = k + 1 + bi, j = k + 1 + bj;
    const double *Lik = A + (long long)(i * 64) * ld + k * 64;
    const double *Ljk = A + (long long)(j * 64) * ld + k * 64;
    double *Aij = A + (long long)(i * 64) * ld + j * 64;
    const bool lookahead = blockIdx.x == 0 && k + 1 < nbs;
    if (lookahead) __builtin_amdgcn_s_setprio(3);   // the look-ahead tile leads to the next pivot chain
    // the 16 entries of A_ij this thread updates, loaded while the MFMA runs
    double old[16];
    {
        int n = 0;
        for_each_pos([&](int r, int c) { old[n++] = (i == j && c > r) ? 0.0 : Aij[(long long)r * ld + c]; });
    }
    f64x4 acc[2][2] = {};
    mfma_nt_64_acc(Lik, ld, Ljk, ld, 64, acc, smem_d, smem_d + 64 * LDP);
    __syncthreads();   // the staging buffers are reused below
    double *tile = smem_d;
    int n = 0;
    for_each_acc(acc, [&](int r, int c, double v) {
        const double o = old[n++];
        if (i == j && c > r) return;
        const double nv = o - v;
        Aij[(long long)r * ld + c] = nv;
        if (lookahead) tile[r * LDP + c] = nv;
    });
    if (lookahead) {
        __syncthreads();
#if CHOL_DIAG_HIER
        chol_diag_hier(tile, smem_d + 64 * LDP, Aij, ld, k + 1, Linv, info);
#else
        chol_diag_block(tile, LDP, Aij, ld, k + 1, Linv, info);
#endif
    }
}

// ----------------------------------------------------------------- ensemble-space gain
// Gram of the extra rows E = [D; d*; Y] (mextp x nyp, rows of A from nyp):
// P = E E^T, lower 64 x 64 tiles on FP64 MFMA, split over the probes: grid
// (tiles, ksplit), workgroup (t, z) forms tile t over probes
// [z kc, (z + 1) kc) into its own partial tile, and gram_extra_sum adds the
// ksplit partials of a tile in the order z = 0, 1, ... (without the split
// the six tiles at C3 run 64 K chunks each on six compute units).
// Without a split (the partial tiles would not fit the scratch): P = E E^T
// in one pass over the probes.
__global__ __launch_bounds__(256) void gram_extra(const double *__restrict__ A, int ld, int nyp, int mextp,
                                                  double *__restrict__ P) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    int bi, bj;
    tri_index(blockIdx.x, bi, bj);
    const double *E = A + (long long)nyp * ld;
    f64x4 acc[2][2] = {};
    mfma_nt_64_acc(E + (long long)(bi * 64) * ld, ld, E + (long long)(bj * 64) * ld, ld, nyp, acc, smem_d,
                   smem_d + 64 * LDP);
    for_each_acc(acc, [&](int r, int c, double v) { P[(long long)(bi * 64 + r) * mextp + bj * 64 + c] = v; });
}

__global__ __launch_bounds__(256) void gram_extra_part(const double *__restrict__ A, int ld, int nyp, int kc,
                                                       double *__restrict__ part) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    int bi, bj;
    tri_index(blockIdx.x, bi, bj);
    const double *E = A + (long long)nyp * ld + (long long)blockIdx.y * kc;
    f64x4 acc[2][2] = {};
    mfma_nt_64_acc(E + (long long)(bi * 64) * ld, ld, E + (long long)(bj * 64) * ld, ld, kc, acc, smem_d,
                   smem_d + 64 * LDP);
    double *dst = part + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * 4096;
    for_each_acc(acc, [&](int r, int c, double v) { dst[r * 64 + c] = v; });
}

// grid (tiles, 16): one element of a tile per thread, its partials loaded
// together (z beyond ksplit re-reads the last one and adds zero) and added
// in the order z = 0, 1, ...
constexpr int GRAM_KSPLIT_MAX = 16;

__global__ __launch_bounds__(256) void gram_extra_sum(const double *__restrict__ part, int ntile, int ksplit,
                                                      int mextp, double *__restrict__ P) {
    int bi, bj;
    tri_index(blockIdx.x, bi, bj);
    const int e = blockIdx.y * 256 + threadIdx.x;
    double pv[GRAM_KSPLIT_MAX];
#pragma unroll
    for (int z = 0; z < GRAM_KSPLIT_MAX; ++z) {
        const int zc = z < ksplit ? z : ksplit - 1;
        pv[z] = part[((long long)zc * ntile + blockIdx.x) * 4096 + e];
    }
    double v = 0.0;
#pragma unroll
    for (int z = 0; z < GRAM_KSPLIT_MAX; ++z) v += z < ksplit ? pv[z] : 0.0;
    P[(long long)(bi * 64 + (e >> 6)) * mextp + bj * 64 + (e & 63)] = v;
}

// The small augmented system of the ensemble-space gain, lds x lds with
// the first npm columns to be factored:
//   [ s^2 I + Y^T Y    .  ]   rows 0 .. npm-1 (identity on the padding)
//   [ (Y^T B)^T        0  ]   rows npm + j, j = 0..N (B_j = D_j, B_N = d*)
//   [ I_N              0  ]   rows npm + N + 1 + i
// Its factorisation leaves -(Y^T B)^T ... and, in the identity rows of the
// Schur block, -(s^2 I + Y^T Y)^-1 Y^T B = -Z: the layout the gain
// extraction reads for the N_y x N_y form.  Only the lower triangle and the
// extra rows are written.
__global__ __launch_bounds__(256) void ens_assemble(const double *__restrict__ P, int mextp, int N, int npm, int lds,
                                                    double s2, double *__restrict__ As) {
    const long long tot = (long long)lds * lds;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
         t += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(t / lds), b = (int)(t - (long long)a * lds);
        if (b > a) continue;
        double v = 0.0;
        if (a < npm) {
            if (a < N && b < N) v = P[(long long)(N + 1 + a) * mextp + N + 1 + b] + (a == b ? s2 : 0.0);
            else v = a == b ? 1.0 : 0.0;
        } else if (b < npm) {
            const int e = a - npm;
            if (b < N && e <= N) v = P[(long long)(N + 1 + b) * mextp + e];
            else if (e >= N + 1 && e <= 2 * N) v = (b == e - N - 1) ? 1.0 : 0.0;
        }
        As[t] = v;
    }
}

// ----------------------------------------------------------------- deferred x* column
// With R = s^2 I the x* column of the gain has the exact form
//   z* = Y^T (Y Y^T + s^2 I)^-1 d* = (s^2 I + Y^T Y)^-1 Y^T d*,
// so it can be formed after the fine forecast while the N_y x N_y
// factorisation (run with d* = 0) proceeds.  M^-1 with M = s^2 I + Y^T Y
// comes out of the small augmented system [[M, .], [I, 0]] (lm = 2 npm
// rows) factored for its first npm columns: its Schur block is -M^-1.
//
// Partial Grams over probe chunks: part[c][t] = sum over the probes p of
// chunk c of Y[p][64 bi + r] Y[p][64 bj + q] for the lower tile t = (bi, bj);
// 4 x 4 entries per thread, probes staged 32 at a time through LDS.
__global__ __launch_bounds__(256) void gram_y_partial(const double *__restrict__ Yk, int kdim, int nyp, int pc,
                                                      double *__restrict__ part) {
    __shared__ double sa[32][64], sb[32][64];
    const int t = blockIdx.x, c = blockIdx.y;
    int bi, bj;
    tri_index(t, bi, bj);
    const int r0 = (threadIdx.x >> 4) * 4, q0 = (threadIdx.x & 15) * 4;
    double acc[4][4] = {};
    const int p_begin = c * pc, p_end = min(nyp, p_begin + pc);
    for (int p0 = p_begin; p0 < p_end; p0 += 32) {
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 64; e += 256) {
            const int pp = e >> 6, col = e & 63;
            const bool in = p0 + pp < p_end;
            sa[pp][col] = in ? Yk[(long long)(p0 + pp) * kdim + bi * 64 + col] : 0.0;
            sb[pp][col] = in ? Yk[(long long)(p0 + pp) * kdim + bj * 64 + col] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int pp = 0; pp < 32; ++pp) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sa[pp][r0 + u];
                b[u] = sb[pp][q0 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
    }
    double *out = part + ((long long)c * gridDim.x + t) * 4096;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(r0 + u) * 64 + q0 + v] = acc[u][v];
}

// The small augmented system, lower triangle: rows a < npm hold
// M = s^2 I + Y^T Y (identity on the padding), rows npm + e hold e_e^T in
// the first npm columns and zeros in the Schur block.  The chunk partials
// are summed in chunk order.
__global__ __launch_bounds__(256) void gram_y_assemble(const double *__restrict__ part, int nchunk, int ntile,
                                                       int N, int npm, double s2, double *__restrict__ Mg) {
    const int lm = 2 * npm;
    const long long tot = (long long)lm * lm;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
         t += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(t / lm), b = (int)(t - (long long)a * lm);
        if (b > a) continue;
        double v = 0.0;
        if (a < npm) {
            if (a < N && b < N) {
                const int bi = a >> 6, bj = b >> 6;
                const int tile = bi * (bi + 1) / 2 + bj;
                const double *pp = part + (long long)tile * 4096 + (a & 63) * 64 + (b & 63);
                for (int c = 0; c < nchunk; ++c) v += pp[(long long)c * ntile * 4096];
                if (a == b) v += s2;
            } else {
                v = a == b ? 1.0 : 0.0;
            }
        } else if (b < npm) {
            v = (b == a - npm) ? 1.0 : 0.0;
        }
        Mg[t] = v;
    }
}

// Y^T (y^o - H(x*)) in partial sums over the probe chunks of the Gram:
// part[c][i] for member i.  The chunk's probes are split over the four
// waves (16 consecutive probes per wave at a time) and the wave sums are
// combined in wave order through LDS.
__global__ __launch_bounds__(1024) void xstar_partial(const double *__restrict__ hx, const double *__restrict__ yobs,
                                                      const double *__restrict__ Yk, int kdim, int Ny, int N, int pc,
                                                      double *__restrict__ part) {
    __shared__ double red[4][256];
    const int c = blockIdx.x, i = threadIdx.x & 255, w = threadIdx.x >> 8;
    const int p0 = c * pc, p1 = min(Ny, p0 + pc);
    double acc = 0.0;
    if (i < N) {
        for (int q = p0 + 16 * w; q < p1; q += 64) {
            const int qe = min(q + 16, p1);
#pragma unroll 4
            for (int p = q; p < qe; ++p) acc += Yk[(long long)p * kdim + i] * (yobs[p] - hx[p]);
        }
    }
    red[w][i] = acc;
    __syncthreads();
    if (w == 0 && i < N) part[(long long)c * 256 + i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
}

// z* = M^-1 v with v the chunk sums (in chunk order) and M^-1 = -(Schur
// block of the factored small system Mg, lower triangle), staged in LDS in
// 64-row slabs; written to zstar (zero-padded to npad) and to column N of
// z64.
__global__ __launch_bounds__(256) void xstar_gain(const double *__restrict__ part, int nchunk, int N, int npad,
                                                  const double *__restrict__ Mg, int npm, double *__restrict__ z64,
                                                  double *__restrict__ zstar, const int32_t *__restrict__ info) {
    __shared__ double v[256];
    __shared__ double slab[64][65];
    if (*info != 0) return;
    const int t = threadIdx.x;
    double acc = 0.0;
    if (t < N) {
#pragma unroll 8
        for (int c = 0; c < nchunk; ++c) acc += part[(long long)c * 256 + t];
    }
    v[t] = acc;
    const int lm = 2 * npm;
    const double *S = Mg + (long long)npm * lm + npm;
    double z = 0.0;
    // thread t takes row t of M^-1 against v; the 64 x 64 sub-blocks
    // (rows r0.., columns b0..) are staged one at a time, each entry read from
    // the stored lower triangle
    for (int b0 = 0; b0 < N; b0 += 64) {
        __syncthreads();   // v written; the previous slab is no longer read
        for (int r0 = 0; r0 < npad && r0 < 256; r0 += 64) {
            // 16 loads in flight per thread, unconditional (outside the
            // matrix a valid element is read and zero stored)
            double mv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int e = t + 256 * q;
                const int rr = r0 + (e >> 6), bb = b0 + (e & 63);
                const bool in = rr < N && bb < N;
                const int rc = in ? rr : 0, bc = in ? bb : 0;
                const long long idx = rc >= bc ? (long long)rc * lm + bc : (long long)bc * lm + rc;
                const double m = S[idx];
                mv[q] = in ? m : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int e = t + 256 * q;
                slab[e >> 6][e & 63] = mv[q];
            }
            __syncthreads();
            if (t >= r0 && t < r0 + 64 && t < N) {
                const int bend = min(64, N - b0);
                for (int bb = 0; bb < bend; ++bb) z -= slab[t - r0][bb] * v[b0 + bb];
            }
            __syncthreads();
        }
    }
    if (t < npad) {
        if (t < N) z64[(long long)N * N + t] = z;
        zstar[t] = t < N ? z : 0.0;
    }
}

// ----------------------------------------------------------------- Z from the Schur block
// Z[i][j] = -M[N+1+i][j] with M the trailing block (rows/cols from nyp).
// z64[j][i] = Z[i][j]; zstar[i] = Z[i][N]; zt holds Z^T for the member
// update, zero-padded to npad x npad: FP64 for MENKF_F64 contexts, else a
// BF16 pair (hi = bf16(z), lo = bf16(z - hi)) at zt and zt + npad^2.
template <typename ZT>
__global__ __launch_bounds__(256) void gain_extract(const double *__restrict__ A, int ld, int nyp, int N, int npad,
                                                    double *__restrict__ z64, ZT *__restrict__ zt,
                                                    double *__restrict__ zstar, uint64_t *__restrict__ dcycle) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0 && dcycle) *dcycle += 1;
    if (t >= npad * npad) return;
    const int j = t / npad, i = t - j * npad;
    const double *M = A + (long long)nyp * ld + nyp;
    double z = 0.0;
    if (i < N && j < N) z = -M[(long long)(N + 1 + i) * ld + j];
    if constexpr (sizeof(ZT) == 8) {
        zt[t] = z;
    } else {
        const ZT hi = ZT((float)z);
        zt[t] = hi;
        zt[t + npad * npad] = ZT((float)(z - (double)(float)hi));
    }
    if (i < N && j < N) z64[(long long)j * N + i] = z;
    if (j == 0) {
        const double zs = i < N ? -M[(long long)(N + 1 + i) * ld + N] : 0.0;
        zstar[i] = zs;
        if (i < N) z64[(long long)N * N + i] = zs;
    }
}

// ----------------------------------------------------------------- member update
// x^a(j) = x^(j) + sum_i Xa_i Z[i][j] and delta^C = sum_i Xa_i z*_i, with
// Xa_i = (x^(i) - xbar) / sqrt(N-1) formed on the fly from the members.
// PW points per workgroup (PW * NPAD floats staged in LDS); the output tile
// (members x points) is Zt (NPAD x NPAD, BF16) times Xa (NPAD x 32 points)
// per wave.  With PW < 128 the four waves also split the output member
// tiles between them.
// TERMS = 1: plain BF16 operands.  TERMS = 3: each operand split into a
// BF16 pair v = hi + lo and the product taken as hi*hi + hi*lo + lo*hi, all
// on BF16 MFMA with FP32 accumulation (about FP32 accuracy at no extra
// memory traffic).
template <int NPAD, int TERMS>
__global__ __launch_bounds__(256) void update_bf16(float *__restrict__ X, float *__restrict__ dc,
                                                   const __bf16 *__restrict__ zt, const double *__restrict__ zstar,
                                                   int N, long long npts, float scale,
                                                   const int32_t *__restrict__ info) {
    constexpr int PW = NPAD <= 128 ? 128 : 64;   // points per workgroup
    constexpr int WPP = PW / 32;                 // waves per point set
    constexpr int MSPLIT = 4 / WPP;              // waves sharing one point set
    __shared__ float xs[NPAD * PW];
    __shared__ float meanf[PW];
    if (*info != 0) return;
    const long long p0 = (long long)blockIdx.x * PW;
    const int tid = threadIdx.x;
    // staging: batches of loads in flight together, unconditional (rows and
    // points past the end re-read a valid element, and zero is stored)
    constexpr int NLD = NPAD * PW / 256;
    constexpr int BATCH = NLD % 16 == 0 ? 16 : 8;
    static_assert(NLD % BATCH == 0, "whole batches");
    for (int q0 = 0; q0 < NLD; q0 += BATCH) {
        float v[BATCH];
#pragma unroll
        for (int q = 0; q < BATCH; ++q) {
            const int e = tid + (q0 + q) * 256;
            const int i = e / PW, p = e - i * PW;
            const int ic = i < N ? i : N - 1;
            const long long pc = p0 + p < npts ? p0 + p : npts - 1;
            v[q] = X[(long long)ic * npts + pc];
        }
#pragma unroll
        for (int q = 0; q < BATCH; ++q) {
            const int e = tid + (q0 + q) * 256;
            const int i = e / PW, p = e - i * PW;
            xs[e] = (i < N && p0 + p < npts) ? v[q] : 0.0f;
        }
    }
    __syncthreads();
    if (tid < PW) {
        double m = 0.0;
        for (int i = 0; i < N; ++i) m += (double)xs[i * PW + tid];
        m /= (double)N;
        meanf[tid] = (float)m;
        double d = 0.0;
        const double sc = (double)scale;
        for (int i = 0; i < N; ++i) d += ((double)xs[i * PW + tid] - m) * sc * zstar[i];
        if (p0 + tid < npts) dc[p0 + tid] = (float)d;
    }
    __syncthreads();
    const int w = tid >> 6, l = tid & 63;
    const int pl = (w % WPP) * 32 + (l & 31);
    const int msub = w / WPP;
    const float mp = meanf[pl];
    bf16x8 bfrag[NPAD / 16];
    bf16x8 bfrag_lo[TERMS == 3 ? NPAD / 16 : 1];
#pragma unroll
    for (int ks = 0; ks < NPAD / 16; ++ks) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = ks * 16 + (l >> 5) * 8 + e;
            const float v = k < N ? (xs[k * PW + pl] - mp) * scale : 0.0f;
            const __bf16 hi = (__bf16)v;
            bfrag[ks][e] = hi;
            if constexpr (TERMS == 3) bfrag_lo[ks][e] = (__bf16)(v - (float)hi);
        }
    }
    // Z fragments are fetched KG k-steps at a time, all before their MFMAs
    constexpr int KS = NPAD / 16;
    constexpr int KG = KS % 4 == 0 ? 4 : 2;
#pragma unroll
    for (int mt = msub; mt < NPAD / 32; mt += MSPLIT) {
        f32x16 acc = {};
        const __bf16 *za = zt + (long long)(mt * 32 + (l & 31)) * NPAD + (l >> 5) * 8;
#pragma unroll
        for (int k0 = 0; k0 < KS; k0 += KG) {
            bf16x8 a[KG], alo[TERMS == 3 ? KG : 1];
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                a[g] = *reinterpret_cast<const bf16x8 *>(za + (k0 + g) * 16);
                if constexpr (TERMS == 3) alo[g] = *reinterpret_cast<const bf16x8 *>(za + NPAD * NPAD + (k0 + g) * 16);
            }
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                const int ks = k0 + g;
                if constexpr (TERMS == 3) {
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[g], bfrag[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[g], bfrag_lo[ks], acc, 0, 0, 0);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[g], bfrag[ks], acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int j = mt * 32 + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
            if (j < N && p0 + pl < npts) X[(long long)j * npts + p0 + pl] = xs[j * PW + pl] + acc[e];
        }
    }
}

// The same update with every wave on its own 32 points and no LDS: lane l
// loads point l % 32 of the NPAD / 2 members k = 16 ks + 8 (l / 32) + e
// (ks < NPAD / 16, e < 8), exactly the members of its MFMA B fragments.
// The FP64 mean and delta^C are each lane's sum over its members plus the
// partner lane's (l ^ 32); of the 16 states a lane writes per output tile,
// half are its own loads and half its partner's (one lane swap each).
// Used for NPAD <= 128 (the fragments then fit the registers).
template <int NPAD, int TERMS>
__global__ __launch_bounds__(256, NPAD <= 96 ? 4 : 2) void update_wave(float *__restrict__ X, float *__restrict__ dc,
                                                   const __bf16 *__restrict__ zt, const double *__restrict__ zstar,
                                                   int N, long long npts, float scale,
                                                   const int32_t *__restrict__ info) {
    constexpr int KS = NPAD / 16;
    if (*info != 0) return;
    const int l = threadIdx.x & 63, h = l >> 5;
    const long long pbase = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
    const long long pt = pbase + (l & 31);
    const bool pin = pt < npts;
    const unsigned off0 = (unsigned)(pin ? pt : 0);
    const unsigned off8 = off0 + (unsigned)(8 * h) * (unsigned)npts;
    // loads: member row 16 ks + e is a uniform base, the lane part an
    // offset (the lane's member is 16 ks + e + 8 h); a member past N reads
    // member 16 ks + e (upper half of the wave) or member 0 (both halves)
    // instead, and the value is discarded below
    float v[KS][8];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k0 = ks * 16 + e;
            const float *row = X + (long long)(k0 < N ? k0 : 0) * npts;
            v[ks][e] = row[k0 + 8 < N ? off8 : off0];
        }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (!(ks * 16 + e + 8 * h < N && pin)) v[ks][e] = 0.0f;
    // FP64 mean and delta^C = sum_k (x^(k) - mean) scale z*_k
    double sm = 0.0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) sm += (double)v[ks][e];
    sm += __shfl_xor(sm, 32);
    const double m = sm / (double)N;
    const double sc = (double)scale;
    double d = 0.0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = ks * 16 + e + 8 * h;
            if (k < N) d += ((double)v[ks][e] - m) * sc * zstar[k];
        }
    d += __shfl_xor(d, 32);
    if (h == 0 && pin) dc[pt] = (float)d;
    // B fragments: anomalies (x - mean) scale, as BF16 (and the BF16 residue)
    const float mp = (float)m;
    bf16x8 bfrag[KS];
    bf16x8 bfrag_lo[TERMS == 3 ? KS : 1];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float a = ks * 16 + e + 8 * h < N ? (v[ks][e] - mp) * scale : 0.0f;
            const __bf16 hi = (__bf16)a;
            bfrag[ks][e] = hi;
            if constexpr (TERMS == 3) bfrag_lo[ks][e] = (__bf16)(a - (float)hi);
        }
    constexpr int KG = KS % 4 == 0 ? 4 : 2;
#pragma unroll
    for (int mt = 0; mt < NPAD / 32; ++mt) {
        f32x16 acc = {};
        const __bf16 *za = zt + (long long)(mt * 32 + (l & 31)) * NPAD + h * 8;
#pragma unroll
        for (int k0 = 0; k0 < KS; k0 += KG) {
            bf16x8 a[KG], alo[TERMS == 3 ? KG : 1];
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                a[g] = *reinterpret_cast<const bf16x8 *>(za + (k0 + g) * 16);
                if constexpr (TERMS == 3) alo[g] = *reinterpret_cast<const bf16x8 *>(za + NPAD * NPAD + (k0 + g) * 16);
            }
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                const int ks = k0 + g;
                if constexpr (TERMS == 3) {
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[g], bfrag[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[g], bfrag_lo[ks], acc, 0, 0, 0);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[g], bfrag[ks], acc, 0, 0, 0);
            }
        }
        // element 4 g + i of the tile: member j = 32 mt + 8 g + 4 h + i, i.e.
        // block ks = 2 mt + g / 2 at offset 8 (g & 1) + 4 h + i, which the
        // lane half g & 1 loaded as its v[ks][4 h + i]: the lane's own value
        // when g & 1 == h, otherwise the partner's (every lane sends its
        // v[ks][4 (1 - h) + i], the index its partner needs)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int ks = 2 * mt + (g >> 1);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float mine = h ? v[ks][4 + i] : v[ks][i];
                const float other = __shfl_xor(h ? v[ks][i] : v[ks][4 + i], 32);
                const float x = ((g & 1) == h) ? mine : other;
                const int j = mt * 32 + 8 * g + 4 * h + i;
                if (j < N && pin) X[(long long)j * npts + pt] = x + acc[4 * g + i];
            }
        }
    }
}

// FP64 update for MENKF_F64 contexts, in two passes so that both are
// parallel over points and members alike (the in-place update of member j
// must not overwrite x^(j) while other workgroups still read it for the
// mean):
//   pass 1: A[i][p] = (x^(i)_p - mean_p) / sqrt(N - 1) into the workspace and
//           delta^C_p = sum_i A[i][p] Z*[i];  16 points x 16 member groups per
//           workgroup, partial sums combined in LDS in a fixed order;
//   pass 2: x^(j)_p += sum_i A[i][p] Z[i, j];  64 points x 4 member groups per
//           workgroup and one j per grid row (Z[., j] read as scalars).
constexpr int UPD_GRP = 16;

__global__ __launch_bounds__(256) void update_anom_f64(const double *__restrict__ X, double *__restrict__ A,
                                                       double *__restrict__ dc, const double *__restrict__ zstar,
                                                       int N, long long npts, double scale,
                                                       const int32_t *__restrict__ info) {
    __shared__ double part[UPD_GRP][UPD_GRP + 1];
    __shared__ double mean[UPD_GRP];
    if (*info != 0) return;
    const int pl = threadIdx.x & (UPD_GRP - 1), g = threadIdx.x / UPD_GRP;
    const long long p = (long long)blockIdx.x * UPD_GRP + pl;
    const bool ok = p < npts;
    double s = 0.0;
    if (ok)
        for (int i = g; i < N; i += UPD_GRP) s += X[(long long)i * npts + p];
    part[g][pl] = s;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int k = 0; k < UPD_GRP; ++k) t += part[k][pl];
        mean[pl] = t / (double)N;
    }
    __syncthreads();
    const double m = mean[pl];
    double d = 0.0;
    if (ok)
        for (int i = g; i < N; i += UPD_GRP) {
            const double a = (X[(long long)i * npts + p] - m) * scale;
            A[(long long)i * npts + p] = a;
            d += a * zstar[i];
        }
    __syncthreads();   // every read of part[][] (the mean) is done
    part[g][pl] = d;
    __syncthreads();
    if (g == 0 && ok) {
        double t = 0.0;
        for (int k = 0; k < UPD_GRP; ++k) t += part[k][pl];
        dc[p] = t;
    }
}

__global__ __launch_bounds__(256) void update_apply_f64(double *__restrict__ X, const double *__restrict__ A,
                                                        const double *__restrict__ zt, int N, int npad,
                                                        long long npts, const int32_t *__restrict__ info) {
    __shared__ double part[4][64];
    if (*info != 0) return;
    const int pl = threadIdx.x & 63, g = threadIdx.x >> 6;   // g is uniform per wave
    const long long p = (long long)blockIdx.x * 64 + pl;
    const int j = blockIdx.y;
    const double *zj = zt + (long long)j * npad;
    double s0 = 0.0, s1 = 0.0;
    if (p < npts) {
        int i = g;
        for (; i + 4 < N; i += 8) {
            s0 += A[(long long)i * npts + p] * zj[i];
            s1 += A[(long long)(i + 4) * npts + p] * zj[i + 4];
        }
        if (i < N) s0 += A[(long long)i * npts + p] * zj[i];
    }
    part[g][pl] = s0 + s1;
    __syncthreads();
    if (g == 0 && p < npts)
        X[(long long)j * npts + p] += (part[0][pl] + part[1][pl]) + (part[2][pl] + part[3][pl]);
}

// ----------------------------------------------------------------- launchers
static hipError_t set_lds(const void *k, size_t bytes) {
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_observe(const Plan &p, int level, const void *state, int nb, double *y, const int32_t *idx,
                          const int32_t *comp, hipStream_t s) {
    const bool coarse = level == MENKF_COARSE;
    const long long stride = (coarse ? p.nc : p.nf) * p.F;
    dim3 grid((p.Ny + 255) / 256, nb);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(obs_eval<double>, grid, dim3(256), 0, s, (const double *)state, stride, nb,
                           (const double *)nullptr, idx, comp, p.Ny, y, p.Ny, coarse ? 1 : 0, p.dim, p.nx, p.ny,
                           p.cfg.ratio, p.nxc, p.nyc, p.open, p.obs_field);
    else
        hipLaunchKernelGGL(obs_eval<float>, grid, dim3(256), 0, s, (const float *)state, stride, nb,
                           (const float *)nullptr, idx, comp, p.Ny, y, p.Ny, coarse ? 1 : 0, p.dim, p.nx, p.ny,
                           p.cfg.ratio, p.nxc, p.nyc, p.open, p.obs_field);
    return hipGetLastError();
}

// Blocked Cholesky of the first nbs * 64 columns of the ld x ld matrix M
// (lower triangle, row-major), Schur complement on the remaining rows.
// With mark set, the event is recorded on s as soon as every trailing
// update still to be issued has at most mark_tiles tiles (before the first
// launch if that already holds): from there on the block steps are bound by
// the latency of the diagonal factorisations and leave most of the GPU
// idle, which is when a caller forks independent work off this point.
static hipError_t chol_blocked(double *A, int ld, int nbs, double *Linv, int32_t *info, size_t lds, hipStream_t s,
                               hipEvent_t mark = nullptr, int mark_tiles = 0) {
    hipError_t e;
    const int nblk = ld / CHOL_NB;
    auto tiles = [nblk](int k) {
        const int below = nblk - k - 1;
        return below > 0 ? below * (below + 1) / 2 : 0;
    };
    bool marked = false;
    if (mark && tiles(0) <= mark_tiles) {
        if ((e = hipEventRecord(mark, s)) != hipSuccess) return e;
        marked = true;
    }
    hipLaunchKernelGGL(chol_diag, dim3(1), dim3(256), 0, s, A, ld, 0, Linv, info);
    for (int k = 0; k < nbs; ++k) {
        const int below = nblk - k - 1;
        if (below > 0) {
            hipLaunchKernelGGL(chol_panel, dim3(below), dim3(256), lds, s, A, ld, k, (const double *)Linv, info);
            hipLaunchKernelGGL(chol_update, dim3(below * (below + 1) / 2), dim3(256), lds, s, A, ld, k, nbs, Linv,
                               info);
        } else if (k + 1 < nbs) {
            hipLaunchKernelGGL(chol_diag, dim3(1), dim3(256), 0, s, A, ld, k + 1, Linv, info);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (mark && !marked && (k + 1 >= nbs || tiles(k + 1) <= mark_tiles)) {
            if ((e = hipEventRecord(mark, s)) != hipSuccess) return e;
            marked = true;
        }
    }
    return hipSuccess;
}

// Z (and its BF16 pair for the member update) from the Schur block of the
// factored augmented matrix M (ld, first n0 columns factored).
static hipError_t extract_gain(const Plan &p, const double *M, int ld, int n0, char *w, uint64_t *dcycle,
                               hipStream_t s) {
    const int N = p.N;
    const int ge = (p.npad * p.npad + 255) / 256;
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(gain_extract<double>, dim3(ge), dim3(256), 0, s, M, ld, n0, N, p.npad,
                           (double *)(w + p.off_z), (double *)(w + p.off_zt), (double *)(w + p.off_zstar), dcycle);
    else
        hipLaunchKernelGGL(gain_extract<__bf16>, dim3(ge), dim3(256), 0, s, M, ld, n0, N, p.npad,
                           (double *)(w + p.off_z), (__bf16 *)(w + p.off_zt), (double *)(w + p.off_zstar), dcycle);
    return hipGetLastError();
}

// Observation, anomalies, innovations and S (steps 1-4); with defer_xstar
// the x* row is left out (d* = 0 in the factorisation) and, for R = s^2 I,
// the small system of the deferred x* column is assembled from Y.
static hipError_t gain_front(const Plan &p, const void *members, const void *xstar, const double *yobs,
                             uint64_t seed, uint64_t cycle, const double *eps, const int32_t *idx,
                             const int32_t *comp, char *w, hipStream_t s, bool defer_xstar) {
    int32_t *info = (int32_t *)(w + p.off_info);
    double *yraw = (double *)(w + p.off_scratch);
    double *A = (double *)(w + p.off_a);
    double *Yk = (double *)(w + p.off_yb);
    const int N = p.N;
    const long long stride = p.nc * p.F;
    const bool f64 = p.cfg.precision == MENKF_F64;
    const int sample = p.cfg.gain_mode == MENKF_GAIN_SAMPLE_EE ? 1 : 0;
    const double rdiag = p.cfg.obs_sigma * p.cfg.obs_sigma;
    hipError_t e;
    const size_t lds = 2 * 64 * LDP * sizeof(double);
    if ((e = set_lds((const void *)chol_panel, lds)) != hipSuccess) return e;
    if ((e = set_lds((const void *)chol_update, lds)) != hipSuccess) return e;
    if ((e = set_lds((const void *)syrk_f64_mfma, lds)) != hipSuccess) return e;
    // 1. H^C of the members (and of x*)
    dim3 g1((p.Ny + 255) / 256, defer_xstar ? N : N + 1);
    if (f64)
        hipLaunchKernelGGL(obs_eval<double>, g1, dim3(256), 0, s, (const double *)members, stride, N,
                           (const double *)xstar, idx, comp, p.Ny, yraw, p.nyp, 1, p.dim, p.nx, p.ny, p.cfg.ratio,
                           p.nxc, p.nyc, p.open, p.obs_field);
    else
        hipLaunchKernelGGL(obs_eval<float>, g1, dim3(256), 0, s, (const float *)members, stride, N,
                           (const float *)xstar, idx, comp, p.Ny, yraw, p.nyp, 1, p.dim, p.nx, p.ny, p.cfg.ratio,
                           p.nxc, p.nyc, p.open, p.obs_field);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // 2. clear the Schur block, reset status
    hipLaunchKernelGGL(zero_extra, dim3(256), dim3(256), 0, s, A, p.ld, p.nyp, p.mext, info);
    // 3. anomalies, innovations, perturbations (FP64)
    const uint64_t *dcycle = cycle == MENKF_CYCLE_DEVICE ? (const uint64_t *)(w + p.off_info + 64) : nullptr;
    hipLaunchKernelGGL(obs_pack, dim3((p.nyp + 15) / 16), dim3(256), 0, s, yraw, p.nyp, N, p.Ny, p.nyp, yobs, eps,
                       seed, cycle, dcycle, p.cfg.obs_sigma, sample, Yk, p.kdim, A, p.ld, defer_xstar ? 0 : 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p.cfg.gain_mode == MENKF_GAIN_ENSEMBLE_SPACE) return hipSuccess;
    // 4. S = Y Y^T + R (+ identity on the padding), FP64 MFMA
    const int nbs = p.nyp / CHOL_NB;
    hipLaunchKernelGGL(syrk_f64_mfma, dim3(nbs * (nbs + 1) / 2), dim3(256), lds, s, (const double *)Yk, p.kdim, p.Ny,
                       sample ? 0.0 : rdiag, A, p.ld);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipSuccess;
}

// Factorisation and the gain factors (steps 5-6).
static hipError_t gain_back(const Plan &p, uint64_t cycle, char *w, hipStream_t s, bool advance_cycle,
                            hipEvent_t mark = nullptr, int mark_tiles = 0) {
    int32_t *info = (int32_t *)(w + p.off_info);
    double *A = (double *)(w + p.off_a);
    double *Linv = (double *)(w + p.off_linv);
    uint64_t *dcycle = (cycle == MENKF_CYCLE_DEVICE && advance_cycle) ? (uint64_t *)(w + p.off_info + 64) : nullptr;
    const size_t lds = 2 * 64 * LDP * sizeof(double);
    hipError_t e;
    if (p.cfg.gain_mode == MENKF_GAIN_ENSEMBLE_SPACE) {
        // 4'. P = E E^T of the extra rows, then the N_e x N_e system
        double *P = (double *)(w + p.off_p), *As = (double *)(w + p.off_as);
        const int mb = p.mextp / CHOL_NB, ntile = mb * (mb + 1) / 2;
        // the probe range is split so that the partial tiles fit the
        // observation scratch, which obs_pack has consumed by now
        size_t cap = (size_t)(p.N + 1) * p.nyp * 8;
        if (cap < 4096 * 8) cap = 4096 * 8;
        int ks = 1;
        for (int c = GRAM_KSPLIT_MAX; c > 1; c /= 2)
            if ((p.nyp / 64) % c == 0 && (size_t)c * ntile * 4096 * 8 <= cap) {
                ks = c;
                break;
            }
        if (ks == 1) {
            if ((e = set_lds((const void *)gram_extra, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(gram_extra, dim3(ntile), dim3(256), lds, s, (const double *)A, p.ld, p.nyp, p.mextp,
                               P);
        } else {
            if ((e = set_lds((const void *)gram_extra_part, lds)) != hipSuccess) return e;
            double *part = (double *)(w + p.off_scratch);
            hipLaunchKernelGGL(gram_extra_part, dim3(ntile, ks), dim3(256), lds, s, (const double *)A, p.ld, p.nyp,
                               p.nyp / ks, part);
            hipLaunchKernelGGL(gram_extra_sum, dim3(ntile, 16), dim3(256), 0, s, (const double *)part, ntile, ks,
                               p.mextp, P);
        }
        hipLaunchKernelGGL(ens_assemble, dim3(256), dim3(256), 0, s, (const double *)P, p.mextp, p.N, p.npm, p.lds,
                           p.cfg.obs_sigma * p.cfg.obs_sigma, As);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = chol_blocked(As, p.lds, p.npm / CHOL_NB, Linv, info, lds, s)) != hipSuccess) return e;
        return extract_gain(p, As, p.lds, p.npm, w, dcycle, s);
    }
    // 5. blocked Cholesky of the first nyp columns, Schur complement on the rest
    if ((e = chol_blocked(A, p.ld, p.nyp / CHOL_NB, Linv, info, lds, s, mark, mark_tiles)) != hipSuccess) return e;
    // 6. Z
    return extract_gain(p, A, p.ld, p.nyp, w, dcycle, s);
}

hipError_t launch_gain(const Plan &p, const void *members, const void *xstar, const double *yobs, uint64_t seed,
                       uint64_t cycle, const double *eps, const int32_t *idx, const int32_t *comp, void *ws,
                       hipStream_t s, bool advance_cycle) {
    char *w = (char *)ws;
    hipError_t e = gain_front(p, members, xstar, yobs, seed, cycle, eps, idx, comp, w, s, false);
    if (e != hipSuccess) return e;
    return gain_back(p, cycle, w, s, advance_cycle);
}

hipError_t launch_gain_deferred_front(const Plan &p, const void *members, const double *yobs, uint64_t seed,
                                      uint64_t cycle, const int32_t *idx, const int32_t *comp, void *ws,
                                      hipStream_t s) {
    if (!p.defer_ok) return hipErrorInvalidValue;
    return gain_front(p, members, nullptr, yobs, seed, cycle, nullptr, idx, comp, (char *)ws, s, true);
}

hipError_t launch_gain_deferred_back(const Plan &p, uint64_t cycle, void *ws, hipStream_t s, hipEvent_t mark,
                                     int mark_tiles) {
    return gain_back(p, cycle, (char *)ws, s, true, mark, mark_tiles);
}

hipError_t launch_xstar_factor(const Plan &p, void *ws, hipStream_t s) {
    char *w = (char *)ws;
    const size_t lds = 2 * 64 * LDP * sizeof(double);
    // M = s^2 I + Y^T Y from the FP64 anomalies (untouched by the N_y x N_y
    // factorisation running beside), in the small augmented system
    const int nt = p.npm / CHOL_NB, ntile = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(gram_y_partial, dim3(ntile, p.gchunks), dim3(256), 0, s, (const double *)(w + p.off_yb),
                       p.kdim, p.nyp, p.gpc, (double *)(w + p.off_gpart));
    hipLaunchKernelGGL(gram_y_assemble, dim3(64), dim3(256), 0, s, (const double *)(w + p.off_gpart), p.gchunks,
                       ntile, p.N, p.npm, p.cfg.obs_sigma * p.cfg.obs_sigma, (double *)(w + p.off_mg));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return chol_blocked((double *)(w + p.off_mg), 2 * p.npm, p.npm / CHOL_NB, (double *)(w + p.off_mlinv),
                        (int32_t *)(w + p.off_info), lds, s);
}

hipError_t launch_xstar_gain(const Plan &p, const void *xstar, const double *yobs, const int32_t *idx,
                             const int32_t *comp, void *ws, hipStream_t s) {
    char *w = (char *)ws;
    double *hx = (double *)(w + p.off_scratch) + (long long)p.N * p.nyp;
    dim3 g1((p.Ny + 255) / 256, 1);
    if (p.cfg.precision == MENKF_F64)
        hipLaunchKernelGGL(obs_eval<double>, g1, dim3(256), 0, s, (const double *)nullptr, 0LL, 0,
                           (const double *)xstar, idx, comp, p.Ny, hx, p.nyp, 1, p.dim, p.nx, p.ny, p.cfg.ratio,
                           p.nxc, p.nyc, p.open, p.obs_field);
    else
        hipLaunchKernelGGL(obs_eval<float>, g1, dim3(256), 0, s, (const float *)nullptr, 0LL, 0,
                           (const float *)xstar, idx, comp, p.Ny, hx, p.nyp, 1, p.dim, p.nx, p.ny, p.cfg.ratio,
                           p.nxc, p.nyc, p.open, p.obs_field);
    double *part = (double *)(w + p.off_gpart);   // the Gram partials are consumed by now
    hipLaunchKernelGGL(xstar_partial, dim3(p.gchunks), dim3(1024), 0, s, (const double *)hx, yobs,
                       (const double *)(w + p.off_yb), p.kdim, p.Ny, p.N, p.gpc, part);
    hipLaunchKernelGGL(xstar_gain, dim3(1), dim3(256), 0, s, (const double *)part, p.gchunks, p.N, p.npad,
                       (const double *)(w + p.off_mg), p.npm, (double *)(w + p.off_z), (double *)(w + p.off_zstar),
                       (const int32_t *)(w + p.off_info));
    return hipGetLastError();
}



hipError_t launch_get_gain(const Plan &p, double *z, void *ws, hipStream_t s) {
    return hipMemcpyAsync(z, (char *)ws + p.off_z, sizeof(double) * (size_t)(p.N + 1) * p.N,
                          hipMemcpyDeviceToDevice, s);
}

template <int NPAD>
static void launch_update_np(const Plan &p, dim3 grid, hipStream_t s, float *X, float *dc, const __bf16 *zt,
                             const double *zs, long long npts, float scale, const int32_t *info) {
    if constexpr (NPAD <= 128) {
        // 128 points per workgroup, as the staged kernel's grid
        if (p.cfg.anomaly_terms == 1)
            hipLaunchKernelGGL((update_wave<NPAD, 1>), grid, dim3(256), 0, s, X, dc, zt, zs, p.N, npts, scale, info);
        else
            hipLaunchKernelGGL((update_wave<NPAD, 3>), grid, dim3(256), 0, s, X, dc, zt, zs, p.N, npts, scale, info);
        return;
    }
    if (p.cfg.anomaly_terms == 1)
        hipLaunchKernelGGL((update_bf16<NPAD, 1>), grid, dim3(256), 0, s, X, dc, zt, zs, p.N, npts, scale, info);
    else
        hipLaunchKernelGGL((update_bf16<NPAD, 3>), grid, dim3(256), 0, s, X, dc, zt, zs, p.N, npts, scale, info);
}

hipError_t launch_update(const Plan &p, void *members, void *dc, void *ws, hipStream_t s) {
    char *w = (char *)ws;
    const int32_t *info = (const int32_t *)(w + p.off_info);
    const long long npts = p.nc * p.F;
    const int N = p.N;
    if (p.cfg.precision == MENKF_F64) {
        // the anomalies go to the coarse Runge-Kutta scratch (N x npts, idle between forecasts)
        double *A = (double *)(w + p.off_c1);
        hipLaunchKernelGGL(update_anom_f64, dim3((unsigned)((npts + UPD_GRP - 1) / UPD_GRP)), dim3(256), 0, s,
                           (const double *)members, A, (double *)dc, (const double *)(w + p.off_zstar), N, npts,
                           1.0 / sqrt((double)(N - 1)), info);
        hipLaunchKernelGGL(update_apply_f64, dim3((unsigned)((npts + 63) / 64), (unsigned)N), dim3(256), 0, s,
                           (double *)members, (const double *)A, (const double *)(w + p.off_zt), N, p.npad, npts,
                           info);
        return hipGetLastError();
    }
    const int pw = p.npad <= 128 ? 128 : 64;
    const dim3 grid((unsigned)((npts + pw - 1) / pw));
    const float scale = (float)(1.0 / sqrt((double)(N - 1)));
    const __bf16 *zt = (const __bf16 *)(w + p.off_zt);
    const double *zs = (const double *)(w + p.off_zstar);
    float *X = (float *)members;
    float *D = (float *)dc;
    switch (p.npad) {
        case 32: launch_update_np<32>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        case 64: launch_update_np<64>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        case 96: launch_update_np<96>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        case 128: launch_update_np<128>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        case 160: launch_update_np<160>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        case 192: launch_update_np<192>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        case 224: launch_update_np<224>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        case 256: launch_update_np<256>(p, grid, s, X, D, zt, zs, npts, scale, info); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace menkf

// Test hook: the 64x64 diagonal-block factorisation alone, one workgroup:
// A (64 x 64, row-major, lower triangle read) -> L (lower, row stride 64),
// Linv (64 x 64), info (0 or 1 + the first non-positive pivot); which = 0
// the pivot sweep, 1 the hierarchical form.  stamps (nullptr or 32 words)
// receive the shader clock at the hierarchical form's phase boundaries.
namespace menkf {
__global__ __launch_bounds__(256) void diag_test_kernel(int which, const double *A, double *L, double *Linv,
                                                        int32_t *info, long long *stamps) {
    __shared__ __attribute__((aligned(16))) double Wd[64 * LDP];
    __shared__ __attribute__((aligned(16))) double scr[DIAG_SCRATCH];
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        if (c <= r) Wd[r * LDP + c] = A[e];
    }
    __syncthreads();
    const long long t0 = (long long)__builtin_amdgcn_s_memtime();
    if (which == 1)
        chol_diag_hier(Wd, scr, L, 64, 0, Linv, info, stamps);
    else
        chol_diag_block(Wd, LDP, L, 64, 0, Linv, info);
    __syncthreads();
    if (stamps && threadIdx.x == 0) {
        stamps[30] = t0;
        stamps[31] = (long long)__builtin_amdgcn_s_memtime();
    }
}
}  // namespace menkf

extern "C" int menkf_test_chol_diag(int which, const double *A, double *L, double *Linv, int32_t *info,
                                    long long *stamps, void *stream) {
    if (which != 0 && which != 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(menkf::diag_test_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, which, A, L, Linv, info,
                       stamps);
    return (int)hipGetLastError();
}

// Test hook: Philox4x32-10 on n (counter, key) sextuples, device pointers.
extern "C" int menkf_test_philox(const uint32_t *in_dev, uint32_t *out_dev, int n, void *stream) {
    hipLaunchKernelGGL(menkf::philox_test_kernel, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, in_dev,
                       out_dev, n);
    return (int)hipGetLastError();
}

// Test hook: one MFMA with the operand/result lane mapping the kernels above
// rely on.  which = 0: A 32x16 BF16, B 16x32 BF16 (row-major) -> C 32x32 FP32;
// which = 1: A 16x4 FP64, B 4x16 FP64 -> C 16x16 FP64.  One wave.
namespace menkf {
__global__ __launch_bounds__(64) void mfma_test_bf16(const __bf16 *a, const __bf16 *b, float *out) {
    const int l = threadIdx.x;
    bf16x8 av, bv;
    for (int e = 0; e < 8; ++e) {
        av[e] = a[(l & 31) * 16 + (l >> 5) * 8 + e];
        bv[e] = b[((l >> 5) * 8 + e) * 32 + (l & 31)];
    }
    f32x16 acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    for (int e = 0; e < 16; ++e) out[(8 * (e >> 2) + 4 * (l >> 5) + (e & 3)) * 32 + (l & 31)] = acc[e];
}
__global__ __launch_bounds__(64) void mfma_test_bf16_16(const __bf16 *a, const __bf16 *b, float *out) {
    const int l = threadIdx.x;
    bf16x8 av, bv;
    for (int e = 0; e < 8; ++e) {
        av[e] = a[(l & 15) * 32 + (l >> 4) * 8 + e];
        bv[e] = b[((l >> 4) * 8 + e) * 16 + (l & 15)];
    }
    f32x4 acc = {};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    for (int e = 0; e < 4; ++e) out[(4 * (l >> 4) + e) * 16 + (l & 15)] = acc[e];
}
__global__ __launch_bounds__(64) void mfma_test_f64(const double *a, const double *b, double *out) {
    const int l = threadIdx.x;
    f64x4 acc = {};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[(l & 15) * 4 + (l >> 4)], b[(l >> 4) * 16 + (l & 15)], acc, 0, 0, 0);
    for (int e = 0; e < 4; ++e) out[(4 * e + (l >> 4)) * 16 + (l & 15)] = acc[e];
}
}  // namespace menkf

extern "C" int menkf_test_mfma(int which, const void *a, const void *b, void *out, void *stream) {
    if (which == 0)
        hipLaunchKernelGGL(menkf::mfma_test_bf16, dim3(1), dim3(64), 0, (hipStream_t)stream, (const __bf16 *)a,
                           (const __bf16 *)b, (float *)out);
    else if (which == 1)
        hipLaunchKernelGGL(menkf::mfma_test_f64, dim3(1), dim3(64), 0, (hipStream_t)stream, (const double *)a,
                           (const double *)b, (double *)out);
    else if (which == 2)
        hipLaunchKernelGGL(menkf::mfma_test_bf16_16, dim3(1), dim3(64), 0, (hipStream_t)stream, (const __bf16 *)a,
                           (const __bf16 *)b, (float *)out);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}
