// Score network for learned AMS scores: near-wake features, forward and
// backward of a small CNN on BF16 matrix cores, and Adam.
//
// The paper's conclusion proposes learning the AMS score function; the
// network here maps a 3 x 16 x 16 picture of the near wake (u_x, u_y, rho - 1)
// to one number: three 3x3 convolutions with 32 channels (zero padding,
// ReLU), a global average and a linear read-out.
//
// Every convolution is an implicit GEMM on the BF16 matrix cores: operands
// rounded to nearest-even from FP32, FP32 accumulation.  Forward: one wave
// owns one image and needs no barrier; the layer's weights sit in registers
// as v_mfma_f32_16x16x32_bf16 A fragments (output channels x (tap, input
// channel)), the activations in the wave's LDS tile (16 x 16 pixels, 40
// BF16 per pixel: 32 channels and a pad that spreads sixteen consecutive
// pixels' 16-byte reads over distinct banks), and each output row is
// written back into the tile two rows after it was computed, when no tap
// of a later row reads its input any more.  The first layer (3 channels)
// uses v_mfma_f32_16x16x16_bf16 with four channel slots per tap.  Backward:
// one workgroup (4 waves) per image on v_mfma_f32_16x16x16_bf16 with padded
// 18 x 18 x C tiles and [K][32] weight tables, K = (tap, input channel).
// Weights are staged in BF16 once per call.  Weight gradients are written
// per image and summed in a fixed order afterwards, so every result is
// deterministic.
#include "cnn_kernels.hpp"

namespace lbm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NC = 32;   // channels of every hidden layer
constexpr int PADW = 18; // padded image side
// LDS rows are padded so that the sixteen lanes of a fragment, one pixel (or
// weight row) apart, fall on distinct banks: 32 channels at a stride of 36
constexpr int TS = 36;   // elements per pixel of a 32-channel activation tile
constexpr int WS = 36;   // elements per row of a staged weight table
constexpr int PAD_ELEMS = PADW * PADW * TS;
constexpr int DZT = 260; // elements per channel of a channel-major dZ copy (256 pixels, padded)

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Lane layout of the 16x16x16 BF16 MFMA: lane l supplies A[l % 16][4 (l / 16) + j]
// and B[4 (l / 16) + j][l % 16] (j = 0..3) and receives D[4 (l / 16) + j][l % 16];
// of the 16x16x32 one: A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16]
// (j = 0..7), the same D.

// The three layers' tables wt[k][o] (k = tap * cin + c, zero rows up to kp)
// in BF16, once per call: layer 1 at 0 (kp = 32), layer 2 at 32 * 32, layer 3
// at (32 + 288) * 32; then the A fragments of the forward kernel (o = 16 tile
// + lane % 16; layer 1: tap = 4 k-step + lane / 16, channel slot j (slot 3
// and taps past 8 zero); layers 2 and 3: input channel 8 (lane / 16) + j).
__global__ __launch_bounds__(256) void cnn_stage_weights_kernel(const float* __restrict__ params,
                                                                unsigned short* __restrict__ wt) {
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= CNN_WT_ELEMS) return;
    float v = 0.0f;
    if (e < CNN_TAB_ELEMS) {
        int layer, r;
        if (e < 32 * NC) { layer = 0; r = e; }
        else if (e < (32 + 288) * NC) { layer = 1; r = e - 32 * NC; }
        else { layer = 2; r = e - (32 + 288) * NC; }
        const int cin = layer == 0 ? 3 : NC;
        const float* w = params + (layer == 0 ? CNN_OFF_W1 : (layer == 1 ? CNN_OFF_W2 : CNN_OFF_W3));
        const int k = r / NC, o = r - k * NC;
        if (k < 9 * cin) {
            const int tap = k / cin, c = k - tap * cin;
            v = w[(o * cin + c) * 9 + tap];
        }
    } else if (e < CNN_FRAG_OFF + CNN_FRAG1_ELEMS) {
        const int r = e - CNN_FRAG_OFF;
        const int j = r & 3, lane = (r >> 2) & 63, mt = (r >> 8) & 1, ks = r >> 9;
        const int o = 16 * mt + (lane & 15), tap = 4 * ks + (lane >> 4);
        if (tap < 9 && j < 3) v = params[CNN_OFF_W1 + (o * 3 + j) * 9 + tap];
    } else {
        const int r0 = e - CNN_FRAG_OFF - CNN_FRAG1_ELEMS;
        const int layer = r0 >= CNN_FRAG23_ELEMS ? 2 : 1;
        const int r = r0 - (layer - 1) * CNN_FRAG23_ELEMS;
        const int j = r & 7, lane = (r >> 3) & 63, mt = (r >> 9) & 1, tap = r >> 10;
        const int o = 16 * mt + (lane & 15), c = 8 * (lane >> 4) + j;
        v = params[(layer == 1 ? CNN_OFF_W2 : CNN_OFF_W3) + (o * NC + c) * 9 + tap];
    }
    wt[e] = f2bf(v);
}

// One staged table (kp rows of 32) into LDS rows of WS elements, 8-byte copies.
__device__ void copy_weights(const unsigned short* __restrict__ src, int kp, unsigned short* wt) {
    const uint2* s2 = (const uint2*)src;
    uint2* d2 = (uint2*)wt;
    for (int e = (int)threadIdx.x; e < kp * NC / 4; e += (int)blockDim.x) d2[(e >> 3) * (WS / 4) + (e & 7)] = s2[e];
}

// n elements (a multiple of 8, 16-byte aligned) set to zero with 16-byte stores.
__device__ void zero_lds(unsigned short* p, int n) {
    uint4* p4 = (uint4*)p;
    for (int e = (int)threadIdx.x; e < n / 8; e += (int)blockDim.x) p4[e] = uint4{0u, 0u, 0u, 0u};
}

// Data gradient of a 32 -> 32 convolution: dX[p][c] = sum_{tap, o} dZ[p - tap + 1][o] W[o][c][tap],
// from the padded dZ tile and the forward weight table (wt[(tap*32 + c)*32 + o]).
__device__ void conv_dgrad(const unsigned short* dz, const unsigned short* wt, f32x4 acc[4][2], int wave, int lane) {
    const int col = lane & 15, kq = (lane >> 4) * 4;
    for (int ks = 0; ks < 9 * NC / 16; ++ks) {
        const int tap0 = (ks * 16) / NC;  // all 16 k of a step share one tap
        const int o0 = ks * 16 + kq - tap0 * NC;  // the lane's 4 consecutive output channels
        bf16x4 bfr[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) bfr[nt] = *(const bf16x4*)(wt + (tap0 * NC + nt * 16 + col) * WS + o0);
        const int dy = tap0 / 3, dx = tap0 - 3 * (tap0 / 3);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int y = wave * 4 + mt;
            const bf16x4 afr = *(const bf16x4*)(dz + ((y - dy + 2) * PADW + (col - dx + 2)) * TS + o0);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = mfma16(afr, bfr[nt], acc[mt][nt]);
        }
    }
}

// Weight gradient of one image: dW[o][c][tap] = sum_p dZ[p][o] X[p + tap - 1][c],
// a GEMM over the 256 pixels; written (not added) to out in canonical order.
// dZ comes channel-major (dzt[o * DZT + p], unpadded pixels): a lane's four
// consecutive pixels of one channel are one 8-byte read.
template <int CIN, int CSTRIDE>
__device__ void conv_wgrad(const unsigned short* dzt, const unsigned short* xin, float* __restrict__ out, int wave,
                           int lane) {
    constexpr int K = 9 * CIN;
    constexpr int KP = (K + 15) / 16 * 16;
    constexpr int TILES = 2 * (KP / 16);
    const int col = lane & 15, kq = (lane >> 4) * 4;
    for (int tile = wave; tile < TILES; tile += 4) {
        const int ot = tile & 1, kt = tile >> 1;
        const int kk = kt * 16 + col;
        const int tap = kk < K ? kk / CIN : 0, c = kk < K ? kk - (kk / CIN) * CIN : 0;
        const int dy = tap / 3, dx = tap - 3 * (tap / 3);
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int py = 0; py < 16; ++py) {
            const bf16x4 afr = *(const bf16x4*)(dzt + (ot * 16 + col) * DZT + py * 16 + kq);
            bf16x4 bfr;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int px = kq + j;
                bfr[j] = kk < K ? (short)xin[((py + dy) * PADW + (px + dx)) * CSTRIDE + c] : (short)0;
            }
            acc = mfma16(afr, bfr, acc);
        }
        if (kk < K) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = ot * 16 + kq + j;
                out[(o * CIN + c) * 9 + tap] = acc[j];
            }
        }
    }
}

// Deterministic per-channel totals of values held in the accumulator layout.
__device__ void channel_sum(const float v[4][2][4], float* red, float* out, int wave, int lane) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        float s = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) s += v[mt][nt][j];
        red[(wave * 4 + (lane >> 4)) * NC + nt * 16 + (lane & 15)] = s;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        float tot = 0.0f;
        for (int q = 0; q < 16; ++q) tot += red[q * NC + threadIdx.x];
        out[threadIdx.x] = tot;
    }
    __syncthreads();
}

// Padded tile of an input image x[b] (FP32 [3][16][16], NCHW) with 4 channel slots.
__device__ void load_input(const float* __restrict__ x, unsigned short* buf) {
    zero_lds(buf, PADW * PADW * 4);
    __syncthreads();
    for (int e = (int)threadIdx.x; e < 3 * 256; e += (int)blockDim.x) {
        const int c = e / 256, p = e - c * 256, y = p / 16, xx = p - y * 16;
        buf[((y + 1) * PADW + (xx + 1)) * 4 + c] = f2bf(x[e]);
    }
}

// Padded tile of a saved activation ([256][32] BF16).
__device__ void load_act(const unsigned short* __restrict__ act, unsigned short* buf) {
    zero_lds(buf, PAD_ELEMS);
    __syncthreads();
    for (int e = (int)threadIdx.x; e < 256 * NC; e += (int)blockDim.x) {
        const int p = e / NC, c = e - p * NC, y = p / 16, xx = p - y * 16;
        buf[((y + 1) * PADW + (xx + 1)) * TS + c] = act[e];
    }
}

__device__ void zero_acc(f32x4 acc[4][2]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

// ---- forward: one wave per image ------------------------------------------

constexpr int TB = 40;  // BF16 elements per pixel of the forward tile (80 bytes)

// One bf16x8 from 16 bytes of LDS.
__device__ __forceinline__ bf16x8 lds_b8(const unsigned short* p) {
    return __builtin_bit_cast(bf16x8, *(const uint4*)p);
}

// Bias, ReLU and BF16 of the lane's output values of one row (two output
// tiles: channels 16 mt + 4 (lane / 16) + j of pixel lane % 16); into the tile
// (8-byte writes) and the saved activation.
__device__ __forceinline__ void fwd_row_out(const f32x4 acc[2], const float bias[2][4], int y, int col, int g,
                                            unsigned short* tile, unsigned short* __restrict__ act, float cs[2][4]) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        ushort4 o;
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = fmaxf(acc[mt][j] + bias[mt][j], 0.0f);
        o.x = f2bf(v[0]);
        o.y = f2bf(v[1]);
        o.z = f2bf(v[2]);
        o.w = f2bf(v[3]);
        const int c0 = 16 * mt + 4 * g;
        if (tile) *(ushort4*)(tile + (y * 16 + col) * TB + c0) = o;
        if (act) *(ushort4*)(act + (y * 16 + col) * NC + c0) = o;
        if (cs) {
#pragma unroll
            for (int j = 0; j < 4; ++j) cs[mt][j] += v[j];
        }
    }
}

// One 32 -> 32 layer of the wave's image, in place in its tile: rows in pairs;
// a pair's outputs are written once the next pair has been computed (the next
// pair's taps read the last row of this pair's inputs; no later pair reads
// them).  A wave's LDS accesses complete in program order, so the writes
// cannot overtake the reads before them.  Taps reaching past the top or bottom row are
// skipped (wave-uniform), past the left or right column read zero.  The last
// layer keeps its outputs out of the tile and sums them per channel (cs).
__device__ __forceinline__ void fwd_layer32(unsigned short* tile, const unsigned short* __restrict__ frag,
                                            const float* __restrict__ bias_p, unsigned short* __restrict__ act,
                                            float cs[2][4], int lane) {
    const int col = lane & 15, g = lane >> 4;
    bf16x8 w[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
            w[t][mt] = __builtin_bit_cast(bf16x8, *(const uint4*)(frag + ((t * 2 + mt) * 64 + lane) * 8));
    float bias[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) bias[mt][j] = bias_p[16 * mt + 4 * g + j];
    unsigned short* const out_tile = cs ? nullptr : tile;
    f32x4 prev[2][2];
    for (int yp = 0; yp < 8; ++yp) {
        const int y0 = 2 * yp;
        f32x4 cur[2][2];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) cur[r][mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            const int px = col + dx;
            const bool inside = px >= 0 && px < 16;
            const int pxc = inside ? px : col;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int ys = y0 + r + dy;
                if (ys < 0 || ys > 15) continue;  // wave-uniform
                bf16x8 v = lds_b8(tile + (ys * 16 + pxc) * TB + 8 * g);
                if (!inside) v = bf16x8{};
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) cur[r][mt] = mfma32(w[t][mt], v, cur[r][mt]);
            }
        }
        if (yp > 0) {  // the previous pair: this pair's taps have read its inputs, later pairs' do not
            fwd_row_out(prev[0], bias, y0 - 2, col, g, out_tile, act, cs);
            fwd_row_out(prev[1], bias, y0 - 1, col, g, out_tile, act, cs);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) prev[r][mt] = cur[r][mt];
    }
    fwd_row_out(prev[0], bias, 14, col, g, out_tile, act, cs);
    fwd_row_out(prev[1], bias, 15, col, g, out_tile, act, cs);
}

__global__ __launch_bounds__(64) void cnn_forward_kernel(CnnArgs a) {
    __shared__ uint4 tile4[256 * TB / 8];  // the activation tile: 16 x 16 pixels x TB
    __shared__ uint2 in2[256];             // the input picture: 16 x 16 pixels x 4 channel slots
    __shared__ float gs[NC];
    unsigned short* const tile = (unsigned short*)tile4;
    const int b = (int)blockIdx.x;
    const int lane = (int)threadIdx.x, col = lane & 15, g = lane >> 4;
    const float* p = a.params;
    unsigned short* const act = a.act ? a.act + (long long)b * 3 * 256 * NC : nullptr;
    // the picture in BF16, pixel-major, channel slot 3 zero
    const float* x = a.x + (long long)b * 3 * 256;
    for (int q = lane; q < 256; q += 64) {
        ushort4 v;
        v.x = f2bf(x[q]);
        v.y = f2bf(x[256 + q]);
        v.z = f2bf(x[512 + q]);
        v.w = 0;
        in2[q] = __builtin_bit_cast(uint2, v);
    }
    __syncthreads();
    // layer 1 (3 -> 32): k = (tap, channel slot), tap = 4 k-step + lane / 16
    {
        const unsigned short* f1 = a.wt + CNN_FRAG_OFF;
        bf16x4 w1[3][2];
#pragma unroll
        for (int ks = 0; ks < 3; ++ks)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
                w1[ks][mt] = __builtin_bit_cast(bf16x4, *(const uint2*)(f1 + ((ks * 2 + mt) * 64 + lane) * 4));
        float bias[2][4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) bias[mt][j] = p[CNN_OFF_B1 + 16 * mt + 4 * g + j];
        for (int y0 = 0; y0 < 16; y0 += 2) {
            f32x4 cur[2][2];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) cur[r][mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 3; ++ks) {
                const int tap = 4 * ks + g;
                const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                const int px = col + dx;
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int ys = y0 + r + dy;
                    const bool ok = tap < 9 && px >= 0 && px < 16 && ys >= 0 && ys < 16;
                    const uint2 raw = in2[ok ? ys * 16 + px : 0];
                    const bf16x4 v = ok ? __builtin_bit_cast(bf16x4, raw) : bf16x4{0, 0, 0, 0};
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) cur[r][mt] = mfma16(w1[ks][mt], v, cur[r][mt]);
                }
            }
            fwd_row_out(cur[0], bias, y0, col, g, tile, act, nullptr);
            fwd_row_out(cur[1], bias, y0 + 1, col, g, tile, act, nullptr);
        }
    }
    __syncthreads();
    fwd_layer32(tile, a.wt + CNN_FRAG_OFF + CNN_FRAG1_ELEMS, p + CNN_OFF_B2, act ? act + 256 * NC : nullptr,
                nullptr, lane);
    __syncthreads();
    float cs[2][4] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
    fwd_layer32(tile, a.wt + CNN_FRAG_OFF + CNN_FRAG1_ELEMS + CNN_FRAG23_ELEMS, p + CNN_OFF_B3,
                act ? act + 2 * 256 * NC : nullptr, cs, lane);
    // per-channel sums over the 16 pixel columns (the lanes of one row of 16), fixed order
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = cs[mt][j];
#pragma unroll
            for (int m = 8; m > 0; m >>= 1) v += __shfl_xor(v, m, 16);
            if (col == 0) gs[16 * mt + 4 * g + j] = v;
        }
    __syncthreads();
    if (lane == 0) {
        float y = p[CNN_OFF_B4];
        for (int o = 0; o < NC; ++o) {
            const float gm = gs[o] * (1.0f / 256.0f);
            if (a.gap) a.gap[(long long)b * NC + o] = gm;
            y += gm * p[CNN_OFF_W4 + o];
        }
        a.y[b] = y;
    }
}

// Backward of one image given the saved activations; writes the image's
// parameter gradients (all but w4, b4) into partial[b][*].
__global__ __launch_bounds__(256) void cnn_backward_kernel(CnnArgs a) {
    __shared__ uint4 bufx_4[PAD_ELEMS / 8];  // 16-byte aligned for the vector LDS reads
    __shared__ uint4 bufd_4[PAD_ELEMS / 8];
    unsigned short* const bufx = (unsigned short*)bufx_4;
    unsigned short* const bufd = (unsigned short*)bufd_4;
    __shared__ uint4 wt4[9 * NC * WS / 8];
    unsigned short* const wt = (unsigned short*)wt4;
    __shared__ float red[16 * NC];
    __shared__ float dsum[NC];
    __shared__ float dg[NC];
    const int b = (int)blockIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int col = lane & 15, kq = (lane >> 4) * 4;
    const float* p = a.params;
    const unsigned short* act = a.act + (long long)b * 3 * 256 * NC;
    float* part = a.partial + (long long)b * CNN_N_PARAMS;
    // dL/dy for the mean squared error, then through the read-out and the average
    const float gy = 2.0f * (a.y[b] - a.labels[b]) / (float)a.batch;
    if (threadIdx.x < NC) dg[threadIdx.x] = gy * p[CNN_OFF_W4 + threadIdx.x] * (1.0f / 256.0f);

    // ---- layer 3: dZ3 = mask(a3) * dG / 256
    load_act(act + 256 * NC, bufx);  // a2, input of layer 3
    copy_weights(a.wt + (32 + 288) * NC, 9 * NC, wt);
    zero_lds(bufd, PAD_ELEMS);
    __syncthreads();
    float vals[4][2][4];
    const unsigned short* a3 = act + 2 * 256 * NC;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int y = wave * 4 + mt, x = kq + j, o = nt * 16 + col;
                const float d = bf2f(a3[(y * 16 + x) * NC + o]) > 0.0f ? dg[o] : 0.0f;
                vals[mt][nt][j] = d;
                bufd[((y + 1) * PADW + (x + 1)) * TS + o] = f2bf(d);
            }
    channel_sum(vals, red, dsum, wave, lane);  // includes the barrier before dZ3 is read
    if (threadIdx.x < NC) part[CNN_OFF_B3 + threadIdx.x] = dsum[threadIdx.x];
    // dZ channel-major for the weight gradient, in the weight table's space once
    // the data gradient has read the table
    auto write_dzt = [&]() {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    wt[(nt * 16 + col) * DZT + (wave * 4 + mt) * 16 + kq + j] = f2bf(vals[mt][nt][j]);
    };
    f32x4 acc[4][2];
    zero_acc(acc);
    conv_dgrad(bufd, wt, acc, wave, lane);
    __syncthreads();
    write_dzt();
    __syncthreads();
    conv_wgrad<NC, TS>(wt, bufx, part + CNN_OFF_W3, wave, lane);
    __syncthreads();  // dZ3 and a2 are read
    // ---- layer 2: dZ2 = mask(a2) * dA2
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int y = wave * 4 + mt, x = kq + j, o = nt * 16 + col;
                const float d = bf2f(bufx[((y + 1) * PADW + (x + 1)) * TS + o]) > 0.0f ? acc[mt][nt][j] : 0.0f;
                vals[mt][nt][j] = d;
                bufd[((y + 1) * PADW + (x + 1)) * TS + o] = f2bf(d);
            }
    channel_sum(vals, red, dsum, wave, lane);
    if (threadIdx.x < NC) part[CNN_OFF_B2 + threadIdx.x] = dsum[threadIdx.x];
    copy_weights(a.wt + 32 * NC, 9 * NC, wt);
    __syncthreads();
    zero_acc(acc);
    conv_dgrad(bufd, wt, acc, wave, lane);
    __syncthreads();
    write_dzt();
    load_act(act, bufx);  // a1 (load_act zeroes then fills; its first barrier orders the reuse)
    __syncthreads();
    conv_wgrad<NC, TS>(wt, bufx, part + CNN_OFF_W2, wave, lane);
    __syncthreads();  // dZ2 and a1's tile are read by the weight gradient
    // ---- layer 1: dZ1 = mask(a1) * dA1, only its weight gradient left (no data gradient)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int y = wave * 4 + mt, x = kq + j, o = nt * 16 + col;
                const float d = bf2f(bufx[((y + 1) * PADW + (x + 1)) * TS + o]) > 0.0f ? acc[mt][nt][j] : 0.0f;
                vals[mt][nt][j] = d;
            }
    write_dzt();
    channel_sum(vals, red, dsum, wave, lane);  // its barriers order dZ1 before the weight gradient
    if (threadIdx.x < NC) part[CNN_OFF_B1 + threadIdx.x] = dsum[threadIdx.x];
    load_input(a.x + (long long)b * 3 * 256, bufx);
    __syncthreads();
    conv_wgrad<3, 4>(wt, bufx, part + CNN_OFF_W1, wave, lane);
}

// Gradients summed over the batch in a fixed order, in two passes: pass 1
// sums each chunk of images in image order (the read-out's own gradients w4,
// b4 from the saved averages) into the chunk's first partial row, pass 2
// sums those rows in chunk order and, in its first workgroup, the loss (a
// fixed-order tree).  Deterministic for a given batch size.  Chunks hold
// about sqrt(batch) images (a power of two, 8 to 256), so that neither pass
// runs a long chain of dependent loads: 16 images at a batch of 256.
__host__ __device__ inline int red_chunk(int batch) {
    int c = 8;
    while (c < 256 && c * c < batch) c *= 2;
    return c;
}

__global__ __launch_bounds__(256) void cnn_reduce_chunks_kernel(CnnArgs a) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= CNN_N_PARAMS) return;
    const int rc = red_chunk(a.batch);
    const int b0 = (int)blockIdx.y * rc, b1 = min(b0 + rc, a.batch);
    float tot = 0.0f;
    if (q >= CNN_OFF_W4) {
        for (int b = b0; b < b1; ++b) {
            const float gy = 2.0f * (a.y[b] - a.labels[b]) / (float)a.batch;
            tot += q == CNN_OFF_B4 ? gy : gy * a.gap[(long long)b * NC + (q - CNN_OFF_W4)];
        }
    } else {
        for (int b = b0; b < b1; ++b) tot += a.partial[(long long)b * CNN_N_PARAMS + q];
    }
    a.partial[(long long)b0 * CNN_N_PARAMS + q] = tot;  // the chunk's first row, read only by this thread
}

__global__ __launch_bounds__(256) void cnn_reduce_final_kernel(CnnArgs a) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int rc = red_chunk(a.batch);
    const int chunks = (a.batch + rc - 1) / rc;
    if (q < CNN_N_PARAMS) {
        float tot = 0.0f;
        for (int c = 0; c < chunks; ++c) tot += a.partial[(long long)c * rc * CNN_N_PARAMS + q];
        a.grads[q] = tot;
    }
    if (blockIdx.x == 0 && a.loss) {  // the whole first workgroup
        __shared__ double red[256];
        double l = 0.0;
        for (int b = (int)threadIdx.x; b < a.batch; b += 256) {
            const double r = (double)a.y[b] - (double)a.labels[b];
            l += r * r;
        }
        red[threadIdx.x] = l;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) *a.loss = (float)(red[0] / a.batch);
    }
}

// Adam (Kingma & Ba) on the FP32 master weights, bias-corrected.
__global__ __launch_bounds__(256) void cnn_adam_kernel(AdamArgs a) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= CNN_N_PARAMS) return;
    const double g = a.grads[q];
    const double m = a.beta1 * a.m[q] + (1.0 - a.beta1) * g;
    const double v = a.beta2 * a.v[q] + (1.0 - a.beta2) * g * g;
    a.m[q] = (float)m;
    a.v[q] = (float)v;
    const double mh = m / (1.0 - pow(a.beta1, (double)a.step));
    const double vh = v / (1.0 - pow(a.beta2, (double)a.step));
    a.params[q] = (float)((double)a.params[q] - a.lr * mh / (sqrt(vh) + a.eps));
}

// Near-wake features of members m0 .. m0+n-1: block = member, thread = pooled pixel.
__global__ __launch_bounds__(256) void features_kernel(FeatureArgs a) {
    const int mi = a.m0 + (int)blockIdx.x;
    const MemberDev m = a.members[mi];
    const int side = a.patch / a.pool;
    const int t = (int)threadIdx.x;
    if (t >= side * side) return;
    const int oy = t / side, ox = t - oy * side;
    const float* st = (a.parity[mi] ? a.pop1 : a.pop0) + m.off;
    const long long plane = (long long)m.nx * m.ny;
    double su = 0.0, sv = 0.0, sr = 0.0;
    for (int yy = 0; yy < a.pool; ++yy)
        for (int xx = 0; xx < a.pool; ++xx) {
            const int y = a.py0 + oy * a.pool + yy, x = a.px0 + ox * a.pool + xx;
            if (in_solid(m, x, y)) continue;  // rho = 1, u = 0 inside a solid
            const long long c = (long long)y * m.nx + x;
            double d[9];
            for (int i = 0; i < 9; ++i) d[i] = (double)st[i * plane + c];
            const double drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
            const double jx = ((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7]);
            const double jy = ((d[2] - d[4]) + (d[5] - d[7])) + (d[6] - d[8]);
            const double rho = 1.0 + drho;
            // post-collision momentum carries the step's force: u = (j - F/2) / rho
            su += (jx - m.half_fx) / rho;
            sv += jy / rho;
            sr += drho;
        }
    const double inv = 1.0 / (double)(a.pool * a.pool);
    float* out = a.out + (long long)blockIdx.x * 3 * side * side;
    out[t] = (float)(su * inv * a.u_scale);
    out[side * side + t] = (float)(sv * inv * a.u_scale);
    out[2 * side * side + t] = (float)(sr * inv * a.rho_scale);
}

hipError_t launch_cnn_forward(const CnnArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(cnn_stage_weights_kernel, dim3((CNN_WT_ELEMS + 255) / 256), dim3(256), 0, st, a.params, a.wt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cnn_forward_kernel, dim3(a.batch), dim3(64), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_cnn_backward(const CnnArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(cnn_backward_kernel, dim3(a.batch), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned cols = (CNN_N_PARAMS + 255) / 256;
    const unsigned chunks = (unsigned)((a.batch + red_chunk(a.batch) - 1) / red_chunk(a.batch));
    hipLaunchKernelGGL(cnn_reduce_chunks_kernel, dim3(cols, chunks), dim3(256), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(cnn_reduce_final_kernel, dim3(cols), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_cnn_adam(const AdamArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(cnn_adam_kernel, dim3((CNN_N_PARAMS + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_features(const FeatureArgs& a, int n, hipStream_t st) {
    hipLaunchKernelGGL(features_kernel, dim3(n), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lbm
