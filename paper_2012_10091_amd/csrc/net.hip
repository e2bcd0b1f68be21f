// Learned convolutional prolongation: inference (fused, BF16 MFMA) and
// training (direct convolutions, BF16 storage, FP32 arithmetic, Adam).
//
// Network: conv3x3(8->32) -> ReLU -> conv3x3(32->32) -> ReLU -> conv3x3(32->4),
// cross-correlation, circular padding on the periodic fine grid.  Input
// channels: Pi_F(delta^C) (4 fields) and x^F_f (4 fields), each mapped to
// (v - in_offset) * in_scale.  The fine correction is
// Pi_F(delta^C) + out / out_scale, so a zero last layer is exactly the plain
// prolongation.
//
// Inference: one workgroup per 16x16 output tile.  The loader computes
// Pi_F(delta^C) on the fly (the same device function as the plain
// prolongation) on the tile plus a halo of 3; the three layers run as
// implicit GEMMs on BF16 MFMA with output channels as the M dimension,
// pixels as N, and K = (tap, input channel) with channels fastest, so each
// lane's 8 K-values are 8 consecutive channels of one tap of one pixel: a
// single 16-byte LDS read from the activations, stored as planes of 8-channel
// chunks.  Layers 1 and 2 use v_mfma_f32_32x32x16_bf16 (32 output channels),
// layer 3 v_mfma_f32_16x16x32_bf16 (4 output channels in a 16-row tile).
#include "common.hpp"

namespace menkf {

// FP32 parameter vector (PyTorch order) and packed BF16 kernel layout.
constexpr int P_W1 = 0, P_B1 = 2304, P_W2 = 2336, P_B2 = 11552, P_W3 = 11584, P_B3 = 12736, P_N = 12740;
constexpr int K_W1 = 0, K_W2 = 2304, K_W3 = 11520, K_N = 20736;

__global__ __launch_bounds__(256) void net_pack_kernel(const float *__restrict__ prm, __bf16 *__restrict__ wk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K_N) return;
    float v;
    if (t < K_W2) {                       // w1 [32][9][8] <- [32][8][3][3]
        const int o = t / 72, rem = t % 72, tap = rem / 8, ic = rem % 8;
        v = prm[P_W1 + o * 72 + ic * 9 + tap];
    } else if (t < K_W3) {                // w2 [32][9][32] <- [32][32][3][3]
        const int u = t - K_W2;
        const int o = u / 288, rem = u % 288, tap = rem / 32, ic = rem % 32;
        v = prm[P_W2 + o * 288 + ic * 9 + tap];
    } else {                              // w3 [32][9][32] <- [4][32][3][3], rows >= 4 zero
        const int u = t - K_W3;
        const int o = u / 288, rem = u % 288, tap = rem / 32, ic = rem % 32;
        v = o < 4 ? prm[P_W3 + o * 288 + ic * 9 + tap] : 0.0f;
    }
    wk[t] = (__bf16)v;
}

// ----------------------------------------------------------------- inference
constexpr int NT = 16, R0 = NT + 6, R1 = NT + 4, R2 = NT + 2;
constexpr int NP0 = R0 * R0, NP1 = R1 * R1, NP2 = R2 * R2, NP3 = NT * NT;

struct NetConst {
    float in_scale[8], in_offset[8], out_scale[4];
    float guard;
};

__device__ __forceinline__ bf16x8 zero_bf16x8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
    return z;
}

// Activations in LDS as channel-chunk planes: the 8 channels of chunk q of
// pixel p (16 bytes, BF16) at byte q * PLANE + 16 p, PLANE = 16 * pixels of
// the layer.  The 32 lanes of an MFMA operand read fetch the same chunk of
// consecutive pixels, i.e. one contiguous 512-byte run (no bank
// conflicts), and every tap of a pixel group is at a compile-time offset
// from one per-lane base address.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <int RIN>
__device__ __forceinline__ constexpr int tap_off(int tap) {   // pixel offset of a 3x3 tap
    return (tap / 3) * RIN + tap % 3;
}

// One conv layer from act_in (IC channels: IC / 8 planes of RIN * RIN
// pixels) to act_out (32 channels: 4 planes of ROUT * ROUT pixels), bias +
// ReLU.  Output channels are the M dimension of v_mfma_f32_32x32x16_bf16,
// 32 pixels the N dimension, K = (tap, input channel) with channels
// fastest.  Each wave takes two 32-pixel groups at a time (nt and nt + 4),
// so two independent accumulator chains interleave on the matrix unit.
template <int IC, int RIN, int ROUT>
__device__ __forceinline__ void conv_layer(const unsigned char *act_in, unsigned char *act_out,
                                           const __bf16 *__restrict__ wk, const float *__restrict__ bias, int wave,
                                           int lane) {
    constexpr int K = 9 * IC;
    constexpr int KCH = (K + 15) / 16;
    constexpr int NPIX = ROUT * ROUT;
    constexpr int PIN = RIN * RIN * 16, POUT = NPIX * 16;
    constexpr int NG = (NPIX + 31) / 32;
    const int half = lane >> 5;
    bf16x8 a[KCH];
#pragma unroll
    for (int ks = 0; ks < KCH; ++ks) {
        const int kb = ks * 16 + half * 8;
        a[ks] = kb < K ? *reinterpret_cast<const bf16x8 *>(wk + (lane & 31) * K + kb) : zero_bf16x8();
    }
    float bv[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) bv[e] = bias[8 * (e >> 2) + 4 * half + (e & 3)];
    for (int nt = wave; nt < NG; nt += 8) {
        const bool two = nt + 4 < NG;   // uniform per wave
        int n[2];
        const unsigned char *src[2];
        bool valid[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            n[h] = (nt + 4 * h) * 32 + (lane & 31);
            valid[h] = n[h] < NPIX;
            const int nn = valid[h] ? n[h] : 0;
            const int py = nn / ROUT, px = nn - py * ROUT;
            // IC = 32: lane half h5 reads chunk 2 (ks & 1) + h5 of tap ks / 2;
            // IC = 8: one plane, lane half h5 reads tap 2 ks + h5
            src[h] = act_in + 16 * (py * RIN + px) + (IC == 32 ? half * PIN : half * 16 * tap_off<RIN>(1));
        }
        f32x16 acc[2] = {{}, {}};
#pragma unroll
        for (int ks = 0; ks < KCH; ++ks) {
            bf16x8 b[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if constexpr (IC == 32) {
                    b[h] = *reinterpret_cast<const bf16x8 *>(src[h] + (ks & 1) * 2 * PIN + 16 * tap_off<RIN>(ks >> 1));
                } else {
                    // taps 2 ks (first half) and 2 ks + 1 (second half, whose base
                    // carries tap_off(1)); the padding tap 9 (zero weights) reads
                    // tap 1's finite values
                    const int t1 = 2 * ks + 1 < 9 ? 2 * ks + 1 : 1;
                    const int o = half ? 16 * (tap_off<RIN>(t1) - tap_off<RIN>(1)) : 16 * tap_off<RIN>(2 * ks);
                    b[h] = *reinterpret_cast<const bf16x8 *>(src[h] + o);
                }
            }
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks], b[0], acc[0], 0, 0, 0);
            if (two) acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks], b[1], acc[1], 0, 0, 0);
        }
        // element e of lane l: channel 8 (e >> 2) + 4 (l >> 5) + (e & 3), pixel
        // l & 31 of the group: 4 consecutive channels of chunk e >> 2, one
        // 8-byte store per chunk
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (valid[h] && (h == 0 || two)) {
                unsigned char *dst = act_out + 16 * n[h] + 8 * half;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    bf16x4 v;
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = (__bf16)fmaxf(acc[h][4 * g + i] + bv[4 * g + i], 0.0f);
                    *reinterpret_cast<bf16x4 *>(dst + g * POUT) = v;
                }
            }
        }
    }
}

__global__ __launch_bounds__(256, 3) void net_prolong_fwd(const float *__restrict__ dc, const float *__restrict__ xf,
                                                       float *__restrict__ xout, const __bf16 *__restrict__ wk,
                                                       const float *__restrict__ prm, NetConst nc, int nx, int ny,
                                                       int r, int nxc, int nyc, int tiles_x, int total_tiles,
                                                       int fallback, int32_t *__restrict__ fb_count,
                                                       int32_t *__restrict__ tile_count,
                                                       const int32_t *__restrict__ info) {
    // LDS in three regions, reused as the layers go (3 workgroups per CU):
    //   A: the input activations in0 and, after them, the coarse window of
    //      delta^C (both dead once layer 1 has run), then layer 2's output act2
    //   B: layer 1's output act1, then (dead after layer 2) the network
    //      output outb and the guard's partial sums
    //   D: the prolonged delta^C at the tile points (read by the epilogue)
    constexpr int CWMAX = 26;   // R0 / r + 5 <= 25 for r >= 1
    constexpr int IN0_B = NP0 * 8 * 2, CWIN_B = 4 * CWMAX * CWMAX * 4, ACT2_B = NP2 * 32 * 2;
    constexpr int REG_A = (IN0_B + CWIN_B > ACT2_B ? IN0_B + CWIN_B : ACT2_B);
    constexpr int ACT1_B = NP1 * 32 * 2, OUTB_B = 4 * NP3 * 4, RED_B = 3 * 4 * 4;
    constexpr int REG_B = (ACT1_B > OUTB_B + RED_B ? ACT1_B : OUTB_B + RED_B);
    static_assert(IN0_B % 16 == 0 && REG_A % 16 == 0 && REG_B % 16 == 0, "16-byte aligned regions");
    __shared__ __align__(16) unsigned char lds_net[REG_A + REG_B + 4 * NP3 * 4];
    __bf16 *in0 = reinterpret_cast<__bf16 *>(lds_net);
    float (*cwin)[CWMAX][CWMAX] = reinterpret_cast<float (*)[CWMAX][CWMAX]>(lds_net + IN0_B);
    unsigned char *act2 = lds_net;
    unsigned char *act1 = lds_net + REG_A;
    float (*outb)[NP3] = reinterpret_cast<float (*)[NP3]>(lds_net + REG_A);
    float (*red)[4] = reinterpret_cast<float (*)[4]>(lds_net + REG_A + OUTB_B);
    float (*dps)[NP3] = reinterpret_cast<float (*)[NP3]>(lds_net + REG_A + REG_B);
    // coarse window of delta^C under the tile + halo 3 (unwrapped coarse
    // origin cx0, cy0; at most CWMAX points per side for r >= 1) and the
    // Lagrange weights of the r sub-positions
    __shared__ float wts[64][4];
    // per fine column (row) of the tile + halo: window column (row) of its
    // first stencil point and its sub-position; periodic coarse column (row)
    // of every window column (row)
    __shared__ int s_bx[R0], s_px[R0], s_by[R0], s_py[R0];
    __shared__ int s_wc[CWMAX], s_wr[CWMAX];
    if (*info != 0) return;
    const int lb = xcd_remap(blockIdx.x, total_tiles);
    const int y0 = (lb / tiles_x) * NT, x0 = (lb % tiles_x) * NT;
    const long long nf = (long long)nx * ny;
    const long long ncp = (long long)nxc * nyc;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // floor division for the (possibly negative) unwrapped coordinates
    auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    const int cx0 = fdiv(x0 - 3, r) - 1, cy0 = fdiv(y0 - 3, r) - 1;
    const int cwx = fdiv(x0 + NT + 2, r) + 3 - cx0, cwy = fdiv(y0 + NT + 2, r) + 3 - cy0;   // <= 25
    if (tid < r) lagrange4<float>(float(tid) / float(r), wts[tid]);
    if (tid < R0) {
        const int X = x0 - 3 + tid, jx = fdiv(X, r);
        s_bx[tid] = jx - 1 - cx0;
        s_px[tid] = X - jx * r;
    } else if (tid >= 64 && tid < 64 + R0) {
        const int Y = y0 - 3 + tid - 64, jy = fdiv(Y, r);
        s_by[tid - 64] = jy - 1 - cy0;
        s_py[tid - 64] = Y - jy * r;
    } else if (tid >= 128 && tid < 128 + CWMAX) {
        s_wc[tid - 128] = wrap(cx0 + tid - 128, nxc);
    } else if (tid >= 192 && tid < 192 + CWMAX) {
        s_wr[tid - 192] = wrap(cy0 + tid - 192, nyc) * nxc;
    }
    // the tile's global reads go out together, before any is used: x^F_f at
    // the thread's (at most two) pixels of the tile + halo and at its output
    // pixel, and the coarse window (32 threads per window row, 8 rows per
    // pass; rows wy = r8 + 8 i, at most CWMAX / 8 + 1 of them)
    // periodic index of a tile + halo coordinate, in [-3, n + 17]: one
    // conditional period on grids of at least 24 points, the full wrap below
    const bool big = nx >= 24 && ny >= 24;
    auto wrapc = [big](int v, int n) { return big ? (v < 0 ? v + n : (v >= n ? v - n : v)) : wrap(v, n); };
    float xin[2][4], xo[4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int p = min(tid + 256 * k, NP0 - 1);
        const int py = p / R0, px = p - py * R0;
        const long long g = (long long)wrapc(y0 - 3 + py, ny) * nx + wrapc(x0 - 3 + px, nx);
#pragma unroll
        for (int f = 0; f < 4; ++f) xin[k][f] = xf[f * nf + g];
    }
    {
        const int py = tid / NT, px = tid - py * NT;
        const long long g = (long long)min(y0 + py, ny - 1) * nx + min(x0 + px, nx - 1);
#pragma unroll
        for (int f = 0; f < 4; ++f) xo[f] = xf[f * nf + g];
    }
    __syncthreads();
    const int c32 = tid & 31, r8 = tid >> 5;
    constexpr int WR = (CWMAX + 7) / 8;
    float wv[4][WR];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int i = 0; i < WR; ++i) {
            const int wy = min(r8 + 8 * i, cwy - 1), wx = min(c32, cwx - 1);
            wv[f][i] = dc[f * ncp + s_wr[wy] + s_wc[wx]];
        }
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int i = 0; i < WR; ++i)
            if (r8 + 8 * i < cwy && c32 < cwx) cwin[f][r8 + 8 * i][c32] = wv[f][i];
    __syncthreads();

    // Pi_F(delta^C) on the tile + halo, separably: the coarse window's rows
    // interpolated in x at the R0 fine columns (sx, in region B: dead before
    // layer 1 writes act1), then in y at every pixel; the products and sums
    // are those of the 4 x 4 form, in the same order
    float (*sx)[CWMAX][R0] = reinterpret_cast<float (*)[CWMAX][R0]>(lds_net + REG_A);
    static_assert(4 * CWMAX * R0 * 4 <= REG_B, "x-interpolated rows fit region B");
    static_assert(R0 <= 32 && CWMAX <= 32, "one window row per 32 threads");
    if (c32 < R0) {
        const float *wx = wts[s_px[c32]];
        const int bx = s_bx[c32];
#pragma unroll
        for (int f = 0; f < 4; ++f)
            for (int wyr = r8; wyr < cwy; wyr += 8) {
                float sa = 0.0f;
#pragma unroll
                for (int b = 0; b < 4; ++b) sa += wx[b] * cwin[f][wyr][bx + b];
                sx[f][wyr][c32] = sa;
            }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int p = tid + 256 * k;
        if (p >= NP0) break;
        const int py = p / R0, px = p - py * R0;
        const float *wy = wts[s_py[py]];
        const int by = s_by[py];
        bf16x8 v;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            float d = 0.0f;
#pragma unroll
            for (int a = 0; a < 4; ++a) d += wy[a] * sx[f][by + a][px];
            const float xv = xin[k][f];
            v[f] = (__bf16)((d - nc.in_offset[f]) * nc.in_scale[f]);
            v[4 + f] = (__bf16)((xv - nc.in_offset[4 + f]) * nc.in_scale[4 + f]);
            if (py >= 3 && py < 3 + NT && px >= 3 && px < 3 + NT) dps[f][(py - 3) * NT + (px - 3)] = d;
        }
        *reinterpret_cast<bf16x8 *>(in0 + p * 8) = v;
    }
    __syncthreads();
    conv_layer<8, R0, R1>(lds_net, act1, wk + K_W1, prm + P_B1, wave, lane);
    __syncthreads();
    conv_layer<32, R1, R2>(act1, act2, wk + K_W2, prm + P_B2, wave, lane);
    __syncthreads();
    {
        // layer 3 (4 output channels) on v_mfma_f32_16x16x32_bf16: M = 16
        // output channels (rows 4..15 of the packed weights are zero), N = 16
        // pixels, K = 32 = the channels of one tap.  Lane l holds A row l % 16
        // and B column l % 16, K values 8 (l / 16) .. 8 (l / 16) + 7; result
        // element i of lane l is channel 4 (l / 16) + i, so lanes 0..15 hold
        // the 4 output channels of their pixel.  Each wave takes two
        // 16-pixel groups at a time.
        bf16x8 a[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            a[tap] = *reinterpret_cast<const bf16x8 *>(wk + K_W3 + (lane & 15) * 288 + tap * 32 + (lane >> 4) * 8);
        constexpr int P2 = NP2 * 16;
        for (int nt = wave; nt < NP3 / 16; nt += 8) {
            int n[2];
            const unsigned char *src[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                n[h] = (nt + 4 * h) * 16 + (lane & 15);
                const int py = n[h] / NT, px = n[h] - py * NT;
                src[h] = act2 + (lane >> 4) * P2 + 16 * (py * R2 + px);
            }
            f32x4 acc[2] = {{}, {}};
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(src[h] + 16 * tap_off<R2>(tap));
                    acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[tap], b, acc[h], 0, 0, 0);
                }
            }
            if (lane < 16) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int f = 0; f < 4; ++f) outb[f][n[h]] = (acc[h][f] + prm[P_B3 + f]) / nc.out_scale[f];
            }
        }
    }
    __syncthreads();
    // epilogue: one thread per output pixel
    const int n = tid;
    const int py = n / NT, px = n - py * NT;
    const int gy = y0 + py, gx = x0 + px;
    float o[4], d[4];
    float s_o = 0.0f, s_d = 0.0f, bad = 0.0f;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        o[f] = outb[f][n];
        d[f] = dps[f][n];
        s_o += o[f] * o[f];
        s_d += d[f] * d[f];
        if (!isfinite(o[f])) bad = 1.0f;
    }
    bool use_net = true;
    if (fallback) {
        // tile sums: within each wave by butterfly shuffles, then over the
        // four waves' partials (one barrier)
        float so = s_o, sd = s_d, sb = bad;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            so += __shfl_xor(so, off);
            sd += __shfl_xor(sd, off);
            sb += __shfl_xor(sb, off);
        }
        if (lane == 0) {
            red[0][wave] = so;
            red[1][wave] = sd;
            red[2][wave] = sb;
        }
        __syncthreads();
        const float no = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const float nd = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        const float nbad = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
        use_net = nbad == 0.0f && isfinite(no) && no <= nc.guard * nc.guard * nd;
        if (!use_net && tid == 0) {
            if (fb_count) atomicAdd(fb_count, 1);
            if (tile_count) atomicAdd(tile_count, 1);
        }
    }
    if (gx < nx && gy < ny) {
        const long long g = (long long)gy * nx + gx;
#pragma unroll
        for (int f = 0; f < 4; ++f) xout[f * nf + g] = xo[f] + d[f] + (use_net ? o[f] : 0.0f);
    }
}

hipError_t launch_net_prolong(const Plan &p, const void *dc, const void *xf, void *xout, const menkf_net *net,
                              int fallback, const int32_t *gate, int32_t *tile_count, hipStream_t s) {
    NetConst nc;
    for (int i = 0; i < 8; ++i) {
        nc.in_scale[i] = net->in_scale[i];
        nc.in_offset[i] = net->in_offset[i];
    }
    for (int i = 0; i < 4; ++i) nc.out_scale[i] = net->out_scale[i];
    nc.guard = net->guard;
    const int tiles_x = (p.nx + NT - 1) / NT, tiles_y = (p.ny + NT - 1) / NT;
    const int total = tiles_x * tiles_y;
    hipLaunchKernelGGL(net_prolong_fwd, dim3(total), dim3(256), 0, s, (const float *)dc, (const float *)xf,
                       (float *)xout, (const __bf16 *)net->wpacked, net->params, nc, p.nx, p.ny, p.cfg.ratio, p.nxc,
                       p.nyc, tiles_x, total, fallback, net->fallback_count_dev, tile_count, gate);
    return hipGetLastError();
}

// ----------------------------------------------------------------- judge
// The plain correction (Pi_F and the relaxed sweeps) judges the network's
// and replaces it when the network strays: a few single-thread kernels
// keep the decision on the device, so a captured cycle replays it.
//   pre:    count the call (not one skipped by its status word); judged
//           call when calls % judge_every == 0;
//           skip the network when the plain correction is kept (stick) and
//           this call is not judged; clear the guarded-tile count
//   mid:    the plain correction is formed when judged, kept, or a tile
//           was guarded
//   decide: on a judged call d = |x_net - x_plain| / |x_plain - x^F_f| in
//           FP64 (fixed-order sums), stick = !(d <= tol); use the plain
//           correction when stick or a tile was guarded
//   select: x^F_a = plain or network correction
__global__ void judge_pre_kernel(const int32_t *__restrict__ info, int32_t *__restrict__ jw, int every) {
    const uint32_t c = (uint32_t)jw[JW_CALLS];
    const int judge = *info == 0 && every > 0 && (c % (uint32_t)every) == 0u;
    if (*info == 0) jw[JW_CALLS] = (int32_t)(c + 1u);
    jw[JW_JUDGE] = judge;
    jw[JW_TILES] = 0;
    jw[JW_SKIP_NET] = (*info != 0 || (jw[JW_STICK] && !judge)) ? 1 : 0;
}

__global__ void judge_mid_kernel(const int32_t *__restrict__ info, int32_t *__restrict__ jw) {
    const int need = jw[JW_JUDGE] || jw[JW_STICK] || jw[JW_TILES] > 0;
    jw[JW_SKIP_PLAIN] = (*info != 0 || !need) ? 1 : 0;
}

__global__ __launch_bounds__(256) void judge_partial(const float *__restrict__ xn, const float *__restrict__ xp,
                                                     const float *__restrict__ xf, long long n,
                                                     const int32_t *__restrict__ jw, double *__restrict__ part) {
    if (jw[JW_SKIP_PLAIN] || !jw[JW_JUDGE]) return;
    __shared__ double s0[256], s1[256];
    double a = 0.0, b = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double p = (double)xp[i];
        const double d = (double)xn[i] - p, c = p - (double)xf[i];
        a += d * d;
        b += c * c;
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ __launch_bounds__(256) void judge_final(const double *__restrict__ part, int nblocks,
                                                   const int32_t *__restrict__ info, int32_t *__restrict__ jw,
                                                   float tol, double *__restrict__ stats) {
    if (*info != 0) return;
    const int judge = jw[JW_JUDGE];
    __shared__ double s[2][256];
    if (judge) {
        double a = 0.0, b = 0.0;
        for (int k = threadIdx.x; k < nblocks; k += 256) {
            a += part[2 * k];
            b += part[2 * k + 1];
        }
        s[0][threadIdx.x] = a;
        s[1][threadIdx.x] = b;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (judge && threadIdx.x < h) {
            s[0][threadIdx.x] += s[0][threadIdx.x + h];
            s[1][threadIdx.x] += s[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (judge) {
        const double a = s[0][0], b = s[1][0];
        const double d = b > 0.0 ? sqrt(a / b) : (a > 0.0 ? INFINITY : 0.0);
        jw[JW_STICK] = (d <= (double)tol) ? 0 : 1;   // NaN fails the test
        if (stats) {
            stats[0] = d;
            stats[1] += 1.0;
        }
    }
    const int tiles = jw[JW_TILES] > 0;
    const int use_plain = jw[JW_STICK] || tiles;
    jw[JW_USE_PLAIN] = use_plain;
    if (stats) {
        stats[2] += (double)use_plain;
        stats[3] += (double)tiles;
    }
}

__global__ __launch_bounds__(256) void judge_select_kernel(const float *__restrict__ xn, const float *__restrict__ xp,
                                                           float *__restrict__ xf, long long n,
                                                           const int32_t *__restrict__ info,
                                                           const int32_t *__restrict__ jw) {
    if (*info != 0) return;
    const float *src = jw[JW_USE_PLAIN] ? xp : xn;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) xf[i] = src[i];
}

__global__ void zero_words_kernel(int32_t *w, int n) {
    if ((int)threadIdx.x < n) w[threadIdx.x] = 0;
}

hipError_t launch_judge_pre(const int32_t *info, int32_t *jw, int judge_every, hipStream_t s) {
    hipLaunchKernelGGL(judge_pre_kernel, dim3(1), dim3(1), 0, s, info, jw, judge_every);
    return hipGetLastError();
}

hipError_t launch_judge_mid(const int32_t *info, int32_t *jw, hipStream_t s) {
    hipLaunchKernelGGL(judge_mid_kernel, dim3(1), dim3(1), 0, s, info, jw);
    return hipGetLastError();
}

hipError_t launch_judge_decide(const Plan &p, const void *xnet, const void *xplain, const void *xf, const int32_t *info,
                               int32_t *jw, float tol, double *judge_dev, void *ws, hipStream_t s) {
    double *part = (double *)((char *)ws + p.off_judge);
    const long long n = (long long)p.F * p.nf;
    long long nb = (n + 255) / 256;
    if (nb > JUDGE_BLOCKS) nb = JUDGE_BLOCKS;
    hipLaunchKernelGGL(judge_partial, dim3((unsigned)nb), dim3(256), 0, s, (const float *)xnet, (const float *)xplain,
                       (const float *)xf, n, (const int32_t *)jw, part);
    hipLaunchKernelGGL(judge_final, dim3(1), dim3(256), 0, s, (const double *)part, (int)nb, info, jw, tol, judge_dev);
    return hipGetLastError();
}

hipError_t launch_judge_select(const Plan &p, const void *xnet, const void *xplain, void *xf, const int32_t *info,
                               const int32_t *jw, hipStream_t s) {
    const long long n = (long long)p.F * p.nf;
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(judge_select_kernel, dim3((unsigned)nb), dim3(256), 0, s, (const float *)xnet,
                       (const float *)xplain, (float *)xf, n, info, jw);
    return hipGetLastError();
}

hipError_t launch_zero_words(int32_t *w, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, w, n);
    return hipGetLastError();
}

hipError_t launch_net_pack(const float *prm, void *wk, hipStream_t s) {
    hipLaunchKernelGGL(net_pack_kernel, dim3((K_N + 255) / 256), dim3(256), 0, s, prm, (__bf16 *)wk);
    return hipGetLastError();
}

// ----------------------------------------------------------------- training
// Crops of C x C output pixels; layer inputs shrink by 2 per valid 3x3
// convolution: input (C+6)^2, a1 (C+4)^2, a2 (C+2)^2, out C^2.  Activations
// BF16, gradients FP32, weights rounded to BF16 on the fly from the FP32
// master copy (the straight-through gradient updates the master copy).
struct TrainShapes {
    int B, C, H0, H1, H2, H3;
};


__global__ __launch_bounds__(256) void train_gather(const float *__restrict__ dproj, const float *__restrict__ xf,
                                                    const float *__restrict__ target, const int32_t *__restrict__ crops,
                                                    int H, int W, TrainShapes sh, NetConst nc,
                                                    __bf16 *__restrict__ in0, float *__restrict__ tgt) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)sh.H0 * sh.H0;
    if (t >= per * sh.B) return;
    const int b = (int)(t / per);
    const int pix = (int)(t - (long long)b * per);
    const int py = pix / sh.H0, px = pix - py * sh.H0;
    const int pr = crops[3 * b], cy = crops[3 * b + 1], cx = crops[3 * b + 2];
    const int gy = wrap(cy - 3 + py, H), gx = wrap(cx - 3 + px, W);
    const long long hw = (long long)H * W;
    const long long g = (long long)pr * 4 * hw + (long long)gy * W + gx;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const float d = dproj[g + f * hw];
        in0[((long long)b * 8 + f) * per + pix] = (__bf16)((d - nc.in_offset[f]) * nc.in_scale[f]);
        in0[((long long)b * 8 + 4 + f) * per + pix] =
            (__bf16)((xf[g + f * hw] - nc.in_offset[4 + f]) * nc.in_scale[4 + f]);
        if (py >= 3 && py < 3 + sh.C && px >= 3 && px < 3 + sh.C) {
            const long long o = ((long long)b * 4 + f) * sh.C * sh.C + (long long)(py - 3) * sh.C + (px - 3);
            tgt[o] = (target[g + f * hw] - d) * nc.out_scale[f];
        }
    }
}

// g = 2 (out - tgt) / n and per-block partial sums of (out - tgt)^2.
__global__ __launch_bounds__(256) void train_mse(const float *__restrict__ out, const float *__restrict__ tgt, long long n,
                                                 float *__restrict__ g, double *__restrict__ part) {
    __shared__ double s[256];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float d = out[i] - tgt[i];
        g[i] = 2.0f * d / (float)n;
        acc += (double)d * d;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// loss = sum of the block partials / n: each lane sums a strided subset,
// then a fixed-order halving over the wave.
__global__ __launch_bounds__(64) void train_loss_final(const double *__restrict__ part, int nb, long long n,
                                                       double *__restrict__ loss) {
    __shared__ double s[64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 64) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s[0] / (double)n;
}

// A valid 3x3 convolution on MFMA for the training passes, from a source
// of Cs <= 32 channels (planes Hs x Hs, NCHW, read with a zero border of
// width pad) to Cd <= 32 channels (planes Hd x Hd, Hd = Hs + 2 pad - 2):
//   forward (MODE CONV_HIDDEN or CONV_LAST, pad 0): the source is BF16,
//     z[o][y][x] = bias[o] + sum_{c,k} bf16(W[o][c][k]) src[c][y+ky][x+kx],
//     dst = bf16(relu(z)) (hidden layers) or z in FP32 (the last layer);
//   data gradient (MODE CONV_DGRAD, pad 2) of a layer with weights
//   W[o][c][k] (o < Cs, c < Cd): the source is the FP32 output gradient,
//   entered as BF16 hi + lo terms, and the taps are flipped,
//     dst[c][y][x] = (act[c][y][x] > 0) sum_{o,k} bf16(W[o][c][8-k]) gpad[o][y+ky][x+kx].
// A workgroup (4 waves) loops over tiles of 4 output rows x 32 columns
// (all Cd channels; wave w takes row w of the tile).  The source tile
// (6 rows x 34 columns x 32 channels) is staged in LDS channel-innermost,
// so that a B fragment (8 channels of one pixel) is one 16-byte read; the
// weight fragments stay in registers for all tiles.  MFMA 32x32x16:
// A[m = output channel][k = source channel], B[k][n = output column].
constexpr int CT_Y = 4, CT_X = 32, CT_SR = CT_Y + 2, CT_SC = CT_X + 2, CT_CP = 40;
enum { CONV_HIDDEN = 0, CONV_LAST = 1, CONV_DGRAD = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void train_conv_mfma(const void *__restrict__ src_, int Cs, int Hs, int pad,
                                                       const float *__restrict__ W, const float *__restrict__ bias,
                                                       int Cd, int Hd, int B, void *__restrict__ dst_,
                                                       const __bf16 *__restrict__ act) {
    constexpr bool BWD = MODE == CONV_DGRAD;
    __shared__ __attribute__((aligned(16))) __bf16 sh[BWD ? 2 : 1][CT_SR * CT_SC * CT_CP];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, h = l >> 5, n = l & 31;
    const int nch = Cs > 16 ? 2 : 1;                 // K chunks of 16 source channels
    // weight fragments: lane row m = n (output channel), K = 16 q + 8 h + e
    bf16x8 wa[2][9];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int cs = 16 * q + 8 * h + e;
                float w = 0.0f;
                if (n < Cd && cs < Cs) w = BWD ? W[(cs * Cd + n) * 9 + 8 - k] : W[(n * Cs + cs) * 9 + k];
                wa[q][k][e] = (__bf16)w;
            }
    const int tilesx = (Hd + CT_X - 1) / CT_X, tilesy = (Hd + CT_Y - 1) / CT_Y;
    const int ntiles = B * tilesy * tilesx;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tx = tile % tilesx, ty = (tile / tilesx) % tilesy, b = tile / (tilesx * tilesy);
        const int x0 = tx * CT_X, y0 = ty * CT_Y;
        __syncthreads();   // the previous tile's reads are done
        for (int i = threadIdx.x; i < 32 * CT_SR * CT_SC; i += 256) {
            const int col = i % CT_SC, rr = (i / CT_SC) % CT_SR, c = i / (CT_SC * CT_SR);
            const int sy = y0 + rr - pad, sx = x0 + col - pad;
            float v = 0.0f;
            if (c < Cs && sy >= 0 && sy < Hs && sx >= 0 && sx < Hs) {
                const long long gi = (((long long)b * Cs + c) * Hs + sy) * Hs + sx;
                if constexpr (BWD)
                    v = ((const float *)src_)[gi];
                else
                    v = (float)((const __bf16 *)src_)[gi];
            }
            const int li = (rr * CT_SC + col) * CT_CP + c;
            const __bf16 hi = (__bf16)v;
            sh[0][li] = hi;
            if constexpr (BWD) sh[BWD ? 1 : 0][li] = (__bf16)(v - (float)hi);
        }
        __syncthreads();
        f32x16 acc = {};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (q < nch) {
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const int li = ((wave + k / 3) * CT_SC + n + k % 3) * CT_CP + 16 * q + 8 * h;
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&sh[0][li]);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[q][k], bv, acc, 0, 0, 0);
                    if constexpr (BWD) {
                        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&sh[BWD ? 1 : 0][li]);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[q][k], bl, acc, 0, 0, 0);
                    }
                }
            }
        }
        // element e: output channel 8 (e / 4) + 4 h + e % 4, column x0 + n
        const int y = y0 + wave, x = x0 + n;
        if (y < Hd && x < Hd) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int m = 8 * (e >> 2) + 4 * h + (e & 3);
                if (m < Cd) {
                    const long long oi = (((long long)b * Cd + m) * Hd + y) * Hd + x;
                    if constexpr (MODE == CONV_DGRAD)
                        ((float *)dst_)[oi] = ((float)act[oi] > 0.0f) ? acc[e] : 0.0f;
                    else if constexpr (MODE == CONV_LAST)
                        ((float *)dst_)[oi] = acc[e] + bias[m];
                    else
                        ((__bf16 *)dst_)[oi] = (__bf16)fmaxf(acc[e] + bias[m], 0.0f);
                }
            }
        }
    }
}

// Weight and bias gradients of a valid 3x3 convolution on MFMA (BF16 in,
// FP32 accumulation): for every tap k = 3 ky + kx
//   C_k[o][c] = sum_{b,y,x} g[b][o][y][x] in[b][c][y + ky][x + kx]
// a 32 x 32 product over the output pixels (Co, Ci <= 32, the rest zero).
// A work item is one 16-pixel run of an output row; the items are split
// evenly over the waves of the grid.  The FP32 gradient enters as two BF16
// terms (hi + lo residue), so the products keep about 16 bits of it.  MFMA
// 32x32x16: lane l holds A[o = l % 32][p = 8 (l / 32) + e] and
// B[p = 8 (l / 32) + e][c = l % 32].  Per workgroup the waves' sums are
// added in LDS in wave order and written as one partial; train_wgrad_reduce
// adds the partials in workgroup order (deterministic).
constexpr int WG_PART = 9 * 1024 + 32;   // floats per workgroup partial: C_k, then the bias sums

__global__ __launch_bounds__(256) void train_wgrad_mfma(const float *__restrict__ g, int Co, int Ho,
                                                        const __bf16 *__restrict__ in, int Ci, int B,
                                                        float *__restrict__ part) {
    __shared__ float red[WG_PART];
    const int Hi = Ho + 2, nxc = (Ho + 15) / 16;
    const long long items = (long long)B * Ho * nxc;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, h = l >> 5, r = l & 31;
    const long long gw = (long long)blockIdx.x * 4 + wave, nw = (long long)gridDim.x * 4;
    const long long i0 = items * gw / nw, i1 = items * (gw + 1) / nw;
    const bool orow = r < Co, ccol = r < Ci;
    f32x16 acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = f32x16{};
    float dbs = 0.0f;
    for (long long it = i0; it < i1; ++it) {
        const int b = (int)(it / ((long long)Ho * nxc));
        const int rem = (int)(it - (long long)b * Ho * nxc);
        const int y = rem / nxc, x0 = 16 * (rem - y * nxc) + 8 * h;
        // A: 8 gradient values of channel o = r (zero past the row or Co)
        const float *gp = g + (((long long)b * Co + (orow ? r : 0)) * Ho + y) * Ho;
        bf16x8 ahi, alo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int x = x0 + e;
            const float v = (orow && x < Ho) ? gp[x < Ho ? x : 0] : 0.0f;
            const __bf16 hi = (__bf16)v;
            ahi[e] = hi;
            alo[e] = (__bf16)(v - (float)hi);
            dbs += v;
        }
        // B: input rows y + ky of channel c = r, 10 values from x0 (zero past the row or Ci)
        const __bf16 *ip = in + (((long long)b * Ci + (ccol ? r : 0)) * Hi + y) * Hi;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            __bf16 v[10];
#pragma unroll
            for (int e = 0; e < 10; ++e) {
                const int x = x0 + e;
                v[e] = (ccol && x < Hi) ? ip[ky * Hi + (x < Hi ? x : 0)] : (__bf16)0.0f;
            }
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                bf16x8 bf;
#pragma unroll
                for (int e = 0; e < 8; ++e) bf[e] = v[e + kx];
                acc[3 * ky + kx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bf, acc[3 * ky + kx], 0, 0, 0);
                acc[3 * ky + kx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bf, acc[3 * ky + kx], 0, 0, 0);
            }
        }
    }
    dbs += __shfl_xor(dbs, 32);
    // the waves' sums into LDS in wave order
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < 9; ++k)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int idx = k * 1024 + (8 * (e >> 2) + 4 * h + (e & 3)) * 32 + r;
                    red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[k][e];
                }
            if (h == 0) red[9 * 1024 + r] = (w == 0 ? 0.0f : red[9 * 1024 + r]) + dbs;
        }
        __syncthreads();
    }
    float *dst = part + (long long)blockIdx.x * WG_PART;
    for (int i = threadIdx.x; i < WG_PART; i += 256) dst[i] = red[i];
}

// dw[(o Ci + c) 9 + k] and db[o] from the workgroup partials: thread j of
// the 8 per output adds partials j, j + 8, ... in order, then the 8 sums are
// added in order (deterministic).
__global__ __launch_bounds__(256) void train_wgrad_reduce(const float *__restrict__ part, int nwg, int Co, int Ci,
                                                          float *__restrict__ dw, float *__restrict__ db) {
    __shared__ float red[8][32];
    const int j = threadIdx.x >> 5, t = blockIdx.x * 32 + (threadIdx.x & 31);
    float s = 0.0f;
    if (t < WG_PART) {
#pragma unroll 8
        for (int w = j; w < nwg; w += 8) s += part[(long long)w * WG_PART + t];
    }
    red[j][threadIdx.x & 31] = s;
    __syncthreads();
    if (j != 0 || t >= WG_PART) return;
    float tot = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) tot += red[k][threadIdx.x];
    if (t < 9 * 1024) {
        const int k = t >> 10, o = (t >> 5) & 31, c = t & 31;
        if (o < Co && c < Ci) dw[(o * Ci + c) * 9 + k] = tot;
    } else if (t - 9 * 1024 < Co) {
        db[t - 9 * 1024] = tot;
    }
}

__global__ __launch_bounds__(256) void train_adam(float *__restrict__ p, const float *__restrict__ g,
                                                  float *__restrict__ m, float *__restrict__ v, int n, float lr,
                                                  float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

struct TrainLayout {
    size_t in0, a1, a2, out, tgt, g3, g2, g1, part, wpart, total;
};

constexpr int WGRAD_WGS = 256;   // workgroups of train_wgrad_mfma

static TrainLayout train_layout(int B, int C) {
    TrainLayout L;
    const size_t H0 = C + 6, H1 = C + 4, H2 = C + 2, H3 = C;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = al256(o + bytes);
        return at;
    };
    L.in0 = take((size_t)B * 8 * H0 * H0 * 2);
    L.a1 = take((size_t)B * 32 * H1 * H1 * 2);
    L.a2 = take((size_t)B * 32 * H2 * H2 * 2);
    L.out = take((size_t)B * 4 * H3 * H3 * 4);
    L.tgt = take((size_t)B * 4 * H3 * H3 * 4);
    L.g3 = take((size_t)B * 4 * H3 * H3 * 4);
    L.g2 = take((size_t)B * 32 * H2 * H2 * 4);
    L.g1 = take((size_t)B * 32 * H1 * H1 * 4);
    L.part = take(1024 * 8);
    L.wpart = take((size_t)WGRAD_WGS * WG_PART * 4);
    L.total = o;
    return L;
}

size_t net_train_workspace(int B, int C) { return train_layout(B, C).total; }

static unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

// workgroups of train_conv_mfma for an output plane of side Hd: one per
// tile, at most 1024 (they loop over the tiles)
static unsigned conv_grid(int B, int Hd) {
    const long long tiles = (long long)B * ((Hd + CT_Y - 1) / CT_Y) * ((Hd + CT_X - 1) / CT_X);
    return (unsigned)(tiles < 1024 ? tiles : 1024);
}

// The training step in three phases sharing the descriptor's workspace:
// forward (layer activations, the loss and its gradient with respect to
// the output), backward (the parameter gradient, from the activations the
// forward phase left) and Adam (the update and the repacked BF16 weights).
enum { TRAIN_FORWARD = 1, TRAIN_BACKWARD = 2, TRAIN_ADAM = 4 };

static hipError_t net_train_phases(const menkf_net_train *t, int phases, hipStream_t s) {
    const TrainLayout L = train_layout(t->batch, t->crop);
    char *w = (char *)t->workspace_dev;
    TrainShapes sh;
    sh.B = t->batch;
    sh.C = t->crop;
    sh.H0 = t->crop + 6;
    sh.H1 = t->crop + 4;
    sh.H2 = t->crop + 2;
    sh.H3 = t->crop;
    NetConst nc;
    for (int i = 0; i < 8; ++i) {
        nc.in_scale[i] = t->in_scale[i];
        nc.in_offset[i] = t->in_offset[i];
    }
    for (int i = 0; i < 4; ++i) nc.out_scale[i] = t->out_scale[i];
    nc.guard = 0.0f;
    __bf16 *in0 = (__bf16 *)(w + L.in0), *a1 = (__bf16 *)(w + L.a1), *a2 = (__bf16 *)(w + L.a2);
    float *out = (float *)(w + L.out), *tgt = (float *)(w + L.tgt), *g3 = (float *)(w + L.g3);
    float *g2 = (float *)(w + L.g2), *g1 = (float *)(w + L.g1);
    double *part = (double *)(w + L.part);
    const float *P = t->params;
    float *G = t->grad;
    const int B = sh.B;
    if (phases & TRAIN_FORWARD) {
        hipLaunchKernelGGL(train_gather, dim3(nblk((long long)sh.H0 * sh.H0 * B)), dim3(256), 0, s, t->dproj, t->xf,
                           t->target, t->crops_dev, t->H, t->W, sh, nc, in0, tgt);
        hipLaunchKernelGGL(train_conv_mfma<CONV_HIDDEN>, dim3(conv_grid(B, sh.H1)), dim3(256), 0, s, (const void *)in0, 8,
                           sh.H0, 0, P + P_W1, P + P_B1, 32, sh.H1, B, (void *)a1, (const __bf16 *)nullptr);
        hipLaunchKernelGGL(train_conv_mfma<CONV_HIDDEN>, dim3(conv_grid(B, sh.H2)), dim3(256), 0, s, (const void *)a1, 32,
                           sh.H1, 0, P + P_W2, P + P_B2, 32, sh.H2, B, (void *)a2, (const __bf16 *)nullptr);
        hipLaunchKernelGGL(train_conv_mfma<CONV_LAST>, dim3(conv_grid(B, sh.H3)), dim3(256), 0, s, (const void *)a2, 32,
                           sh.H2, 0, P + P_W3, P + P_B3, 4, sh.H3, B, (void *)out, (const __bf16 *)nullptr);
        const long long nout = (long long)B * 4 * sh.H3 * sh.H3;
        int nbm = (int)nblk(nout);
        if (nbm > 1024) nbm = 1024;
        hipLaunchKernelGGL(train_mse, dim3(nbm), dim3(256), 0, s, (const float *)out, (const float *)tgt, nout, g3,
                           part);
        hipLaunchKernelGGL(train_loss_final, dim3(1), dim3(64), 0, s, (const double *)part, nbm, nout, t->loss_dev);
    }
    if (phases & TRAIN_BACKWARD) {
        float *wpart = (float *)(w + L.wpart);
        auto wgrad = [&](const float *gout, int Co, int Ho, const __bf16 *act, int Ci, float *dw, float *db) {
            hipLaunchKernelGGL(train_wgrad_mfma, dim3(WGRAD_WGS), dim3(256), 0, s, gout, Co, Ho, act, Ci, B, wpart);
            hipLaunchKernelGGL(train_wgrad_reduce, dim3((WG_PART + 31) / 32), dim3(256), 0, s,
                               (const float *)wpart, WGRAD_WGS, Co, Ci, dw, db);
        };
        // layer 3
        wgrad((const float *)g3, 4, sh.H3, (const __bf16 *)a2, 32, G + P_W3, G + P_B3);
        hipLaunchKernelGGL(train_conv_mfma<CONV_DGRAD>, dim3(conv_grid(B, sh.H2)), dim3(256), 0, s, (const void *)g3, 4,
                           sh.H3, 2, P + P_W3, (const float *)nullptr, 32, sh.H2, B, (void *)g2, (const __bf16 *)a2);
        // layer 2
        wgrad((const float *)g2, 32, sh.H2, (const __bf16 *)a1, 32, G + P_W2, G + P_B2);
        hipLaunchKernelGGL(train_conv_mfma<CONV_DGRAD>, dim3(conv_grid(B, sh.H1)), dim3(256), 0, s, (const void *)g2, 32,
                           sh.H2, 2, P + P_W2, (const float *)nullptr, 32, sh.H1, B, (void *)g1, (const __bf16 *)a1);
        // layer 1
        wgrad((const float *)g1, 32, sh.H1, (const __bf16 *)in0, 8, G + P_W1, G + P_B1);
    }
    if (phases & TRAIN_ADAM) {
        const float c1 = 1.0f - powf(t->beta1, (float)t->step);
        const float c2 = 1.0f - powf(t->beta2, (float)t->step);
        hipLaunchKernelGGL(train_adam, dim3(nblk(P_N)), dim3(256), 0, s, t->params, (const float *)G, t->adam_m,
                           t->adam_v, P_N, t->lr, t->beta1, t->beta2, t->eps, c1, c2);
        if (t->wpacked) return launch_net_pack(t->params, t->wpacked, s);
    }
    return hipGetLastError();
}

hipError_t launch_net_train_step(const menkf_net_train *t, hipStream_t s) {
    return net_train_phases(t, TRAIN_FORWARD | TRAIN_BACKWARD | (t->apply_adam ? TRAIN_ADAM : 0), s);
}

hipError_t launch_net_forward(const menkf_net_train *t, hipStream_t s) { return net_train_phases(t, TRAIN_FORWARD, s); }

hipError_t launch_net_backward(const menkf_net_train *t, hipStream_t s) {
    return net_train_phases(t, TRAIN_BACKWARD, s);
}

hipError_t launch_net_adam(const menkf_net_train *t, hipStream_t s) { return net_train_phases(t, TRAIN_ADAM, s); }

}  // namespace menkf
