// Internal declarations shared by the HIP translation units of libmenkf.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>

#include <type_traits>

#include "../../include/menkf.h"

namespace menkf {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

// Blocks are dispatched round-robin over the 8 XCDs (block i -> XCD i % 8).
// Remap so that each XCD receives one contiguous range of logical blocks:
// neighbouring stencil tiles then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int i, int total) {
    const int xcd = i & 7;
    const int local = i >> 3;
    const int per = total >> 3;
    const int rem = total & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// f(std::integral_constant<int, I>) for I = B .. E-1 in order: the body is
// instantiated once per I, so array indices derived from I are constants.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

__device__ __forceinline__ int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return __float2bfloat16(v); }

// Raw buffer access: a 128-bit resource (base, size in bytes) and 32-bit
// byte offsets, one in a VGPR and one uniform in an SGPR, so per-element
// addressing costs one 32-bit multiply-add instead of 64-bit pointer
// arithmetic.  Accesses outside [0, bytes) read 0 and write nothing.
typedef __amdgpu_buffer_rsrc_t buf_t;
__device__ __forceinline__ buf_t buf_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buf_ld(buf_t r, int voff, int soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_ld(buf_t r, int voff, int soff, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ T buf_load(buf_t r, int voff, int soff) {
    return buf_ld(r, voff, soff, T());
}
__device__ __forceinline__ void buf_store(float v, buf_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(double v, buf_t r, int voff, int soff) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

// Philox4x32-10 (Salmon et al., SC'11): per round the products M0*c0 and
// M1*c2 are split into hi/lo words and the counter becomes
// (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key advances by the Weyl constants
// between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
    }
}

// Standard normal number k of member i at a cycle on a stream: counter
// (k >> 1, i, cycle, stream), key = seed, 53-bit uniforms u = (m + 1/2) 2^-53
// from word pairs, Box-Muller cos branch for even k and sin branch for odd k.
__device__ __forceinline__ double philox_normal(uint64_t seed, uint64_t cycle, int i, int k, uint32_t stream) {
    uint32_t c[4] = {(uint32_t)(k >> 1), (uint32_t)i, (uint32_t)cycle, stream};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) * 0x1p-53;
    const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6) + 0.5) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;
    return (k & 1) ? rad * sin(ang) : rad * cos(ang);
}

// Four-point Lagrange basis on nodes -1, 0, 1, 2 evaluated at s in [0, 1).
template <typename R>
__host__ __device__ __forceinline__ void lagrange4(R s, R w[4]) {
    const R sm1 = s - R(1), sm2 = s - R(2), sp1 = s + R(1);
    w[0] = -s * sm1 * sm2 / R(6);
    w[1] = sp1 * sm1 * sm2 / R(2);
    w[2] = -sp1 * s * sm2 / R(2);
    w[3] = sp1 * s * sm1 / R(6);
}

// Pi_F on an open 1D grid (the inlet-forced case): fine node x uses the
// cubic through coarse nodes b..b+3, b = clamp(x / r - 1, 0, nc - 4), so the
// stencil turns one-sided at both ends.  Writes the weights and returns b.
// In the interior b = x / r - 1 and the weights are those of the periodic
// stencil (lagrange4 is a polynomial in s, valid outside [0, 1) too).
template <typename R>
__host__ __device__ __forceinline__ int open_cubic(int x, int r, int nc, R w[4]) {
    int b = x / r - 1;
    b = b < 0 ? 0 : (b > nc - 4 ? nc - 4 : b);
    lagrange4<R>(R(x - (b + 1) * r) / R(r), w);
    return b;
}

// (Pi_F d)(y, x): cubic Lagrange interpolation of a periodic coarse field
// (nyc x nxc, nyc = 1 in 1D) at fine node (y, x), tensor product in 2D.
template <typename T>
__device__ __forceinline__ T prolong_at(const T *__restrict__ d, int nxc, int nyc, int r, int y, int x) {
    const int jx = x / r, mx = x - jx * r;
    T wx[4];
    lagrange4<T>(T(mx) / T(r), wx);
    if (nyc == 1) {
        T acc = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += wx[b] * d[wrap(jx - 1 + b, nxc)];
        return acc;
    }
    const int jy = y / r, my = y - jy * r;
    T wy[4];
    lagrange4<T>(T(my) / T(r), wy);
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const T *row = d + (long long)wrap(jy - 1 + a, nyc) * nxc;
        T sa = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) sa += wx[b] * row[wrap(jx - 1 + b, nxc)];
        acc += wy[a] * sa;
    }
    return acc;
}

// Derived sizes and workspace offsets of one context.
struct Plan {
    menkf_config cfg;
    int dim, F;
    int nx, ny, nxc, nyc;
    long long nf, nc;          // points per field, fine / coarse
    int N, Ny;                 // members, probes
    int npad;                  // N rounded up to 32 (MFMA tiles)
    int kdim;                  // K of the S product: N or 2N (sample mode), rounded up to 64
    int nyp;                   // Ny rounded up to the Cholesky block
    int mext;                  // extra rows of the augmented factorisation: 2N+1
    int mextp;                 // rounded up to the block
    int ld;                    // leading dimension of the augmented matrix
    size_t tsize;              // sizeof state element
    // workspace offsets (bytes)
    size_t off_info, off_f1, off_f2, off_facc, off_c1, off_c2, off_cacc;
    size_t off_yb, off_a, off_linv, off_z, off_zt, off_zstar, off_scratch;
    // ensemble-space gain: Gram of the extra rows (mextp^2) and the small
    // augmented matrix [[s^2 I + Y^T Y, .], [ (Y^T B)^T ; I ], .] (lds^2)
    int npm, lds;              // N rounded up to the block, npm + mextp
    size_t off_p, off_as;
    size_t ws_bytes;
    menkf_schedule sched[2];   // forecast schedule per level (0 fine, 1 coarse)
    double tuned_ms[2];        // forecast time of the autotuned schedule (0: not tuned)
    int tuned_nsteps[2];       // ... and the window it was timed on
    // inlet-forced model: open grid (one-sided prolongation and observation),
    // the trial member forecast of the parameter filter and its parameters
    int open;
    int obs_field;             // field the 1D observation reads (rho u for the Euler model)
    size_t off_trial, off_thf;
    // deferred x* column (R = s^2 I): small system [[s^2 I + Y^T Y, .], [I, 0]],
    // its Linv scratch, and the chunked partial Grams of Y
    int defer_ok, gchunks, gpc;
    size_t off_mg, off_mlinv, off_gpart;
    // judge of the learned prolongation: partial sums of its distance reduction
    size_t off_judge;
};

// Words of the learned prolongation's judge, in the workspace's status
// block (int32 each, from byte JUDGE_WORDS of the block)
constexpr int JUDGE_WORDS = 128;
enum { JW_CALLS = 0, JW_STICK = 1, JW_TILES = 2, JW_SKIP_NET = 3, JW_SKIP_PLAIN = 4, JW_JUDGE = 5, JW_USE_PLAIN = 6,
       JW_N = 8 };
constexpr int JUDGE_BLOCKS = 512;
// Words of the pipelined cycle (from byte PIPE_WORDS of the status block):
// a correction is pending (left by the last pipelined cycle), and the skip
// word of the deferred correction (no correction pending, or a failure)
constexpr int PIPE_WORDS = 192;
enum { PW_PEND = 0, PW_SKIP = 1, PW_N = 2 };

constexpr int CHOL_NB = 64;

// Kernel launchers (each returns hipError_t of the launch).
// forecast
hipError_t launch_burgers_forecast(const Plan &p, int level, void *state, int nb, int nsteps,
                                   void *prev, void *ws, hipStream_t s);
size_t inlet_window_lds(int n, size_t tsize);
size_t euler_window_lds(int n, size_t tsize);
hipError_t launch_euler_forecast(const Plan &p, int level, void *state, int nb, int nsteps, void *prev,
                                 const double *theta, const double *t0, hipStream_t s);
hipError_t launch_euler_sweep(const Plan &p, const void *x, const void *xp, void *out, double alpha,
                              const int32_t *info, hipStream_t s);
hipError_t launch_inlet_forecast(const Plan &p, int level, void *state, int nb, int nsteps, void *prev,
                                 const double *theta, const double *t0, hipStream_t s);
// dual EnKF parameter filter
hipError_t launch_param_perturb(const Plan &p, const double *theta, double *thf, uint64_t seed, uint64_t cycle,
                                void *ws, hipStream_t s);
hipError_t launch_param_update(const Plan &p, const double *thf, double *tha, double *tmean, void *ws,
                               hipStream_t s);
hipError_t launch_clock_advance(double *clock, double dt_window, hipStream_t s);
hipError_t launch_dual_prep(const Plan &p, const void *members, void *trial, const double *theta, double *thf,
                            uint64_t seed, uint64_t cycle, void *ws, hipStream_t s);
// stencil tile table of the 2D model
int ns_tile_count(int precision);
void ns_tile_shape(int precision, int i, int *tx, int *ty);
int ns_tile_index(int precision, int tx, int ty);   // -1 if not in the table
struct Plan;
// rows per workgroup of the paired row march (two RK stages per launch)
#ifndef PAIR_ROWS_BUILD
#define PAIR_ROWS_BUILD 32
#endif
constexpr int PAIR_ROWS = PAIR_ROWS_BUILD;
bool ns_march_applies(const Plan &p, int level, int rows);   // the 0 x rows row-march schedule runs on this level
hipError_t launch_ns_forecast(const Plan &p, int level, void *state, int nb, int nsteps,
                              void *prev, void *ws, hipStream_t s);
// grids
hipError_t launch_restrict(const Plan &p, const void *xf, void *xc, hipStream_t s);
hipError_t launch_prolong_add(const Plan &p, const void *dc, const void *xin, void *xout,
                              const int32_t *info, hipStream_t s);
hipError_t launch_sweep(const Plan &p, const void *xin, const void *xprev, void *xout,
                        double alpha, const int32_t *info, void *ws, hipStream_t s);
hipError_t launch_copy(const Plan &p, const void *src, void *dst, const int32_t *info, hipStream_t s);
hipError_t launch_recentre(const Plan &p, void *members, const void *xf, const int32_t *info, hipStream_t s);
hipError_t launch_ns_resid(const Plan &p, const void *x, const void *xp, void *out, hipStream_t s);
hipError_t launch_burgers_resid(const Plan &p, const void *x, const void *xp, void *out, hipStream_t s);
// analysis
hipError_t launch_gain(const Plan &p, const void *members, const void *xstar, const double *yobs,
                       uint64_t seed, uint64_t cycle, const double *eps, const int32_t *idx,
                       const int32_t *comp, void *ws, hipStream_t s, bool advance_cycle = true);
hipError_t launch_get_gain(const Plan &p, double *z, void *ws, hipStream_t s);
// the gain with the x* column deferred: front (observation of the members,
// anomalies, S, small system), back (factorisation, Z with z* = 0), the
// small system's factorisation, then z* once x* is known
hipError_t launch_gain_deferred_front(const Plan &p, const void *members, const double *yobs, uint64_t seed,
                                      uint64_t cycle, const int32_t *idx, const int32_t *comp, void *ws,
                                      hipStream_t s);
// The factorisation of the deferred gain; mark is recorded on s once the
// remaining trailing updates have at most mark_tiles tiles each.
hipError_t launch_gain_deferred_back(const Plan &p, uint64_t cycle, void *ws, hipStream_t s, hipEvent_t mark,
                                     int mark_tiles);
hipError_t launch_xstar_factor(const Plan &p, void *ws, hipStream_t s);
hipError_t launch_xstar_gain(const Plan &p, const void *xstar, const double *yobs, const int32_t *idx,
                             const int32_t *comp, void *ws, hipStream_t s);
hipError_t launch_update(const Plan &p, void *members, void *dc, void *ws, hipStream_t s);
hipError_t launch_observe(const Plan &p, int level, const void *state, int nb, double *y,
                          const int32_t *idx, const int32_t *comp, hipStream_t s);
hipError_t launch_diagnostics(const Plan &p, const void *xa, const void *xt, double *out, void *ws, hipStream_t s);
hipError_t launch_spread(const Plan &p, const void *members, int nb, double *out, void *ws, hipStream_t s);
// menkf_diagnostics with its partials in a static device array (no workspace)
hipError_t launch_diagnostics_noalloc(const Plan &p, const void *xa, const void *xt, double *out, hipStream_t s);
size_t diagnostics_noalloc_need(const Plan &p);   // doubles of the array one call uses
size_t diagnostics_noalloc_capacity();              // doubles the array holds
hipError_t launch_set_word(int32_t *w, int32_t v, hipStream_t s);
hipError_t launch_set_word64(uint64_t *w, uint64_t v, hipStream_t s);
hipError_t launch_pipe_skip(const int32_t *info, int32_t *pw, hipStream_t s);
// learned prolongation
// gate: the kernel does nothing when *gate != 0 (the status word, or the
// judge's skip word); tile_count (optional) counts this call's guarded tiles
hipError_t launch_net_prolong(const Plan &p, const void *dc, const void *xf, void *xout, const menkf_net *net,
                              int fallback, const int32_t *gate, int32_t *tile_count, hipStream_t s);
hipError_t launch_net_pack(const float *prm, void *wk, hipStream_t s);
// the judge of LEARNED_FALLBACK (words jw = status block + JUDGE_WORDS)
hipError_t launch_judge_pre(const int32_t *info, int32_t *jw, int judge_every, hipStream_t s);
hipError_t launch_judge_mid(const int32_t *info, int32_t *jw, hipStream_t s);
hipError_t launch_judge_decide(const Plan &p, const void *xnet, const void *xplain, const void *xf, const int32_t *info,
                               int32_t *jw, float tol, double *judge_dev, void *ws, hipStream_t s);
hipError_t launch_judge_select(const Plan &p, const void *xnet, const void *xplain, void *xf, const int32_t *info,
                               const int32_t *jw, hipStream_t s);
hipError_t launch_zero_words(int32_t *w, int n, hipStream_t s);
hipError_t launch_net_train_step(const menkf_net_train *t, hipStream_t s);
hipError_t launch_net_forward(const menkf_net_train *t, hipStream_t s);
hipError_t launch_net_backward(const menkf_net_train *t, hipStream_t s);
hipError_t launch_net_adam(const menkf_net_train *t, hipStream_t s);
size_t net_train_workspace(int B, int C);

}  // namespace menkf
