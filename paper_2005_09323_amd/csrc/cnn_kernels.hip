// Score network for learned AMS scores: near-wake features, forward and
// backward of a small CNN on BF16 matrix cores, and Adam.
//
// The paper's conclusion proposes learning the AMS score function; the
// network here maps a 3 x 16 x 16 picture of the near wake (u_x, u_y, rho - 1)
// to one number: three 3x3 convolutions with 32 channels (zero padding,
// ReLU), a global average and a linear read-out.
//
// Every convolution is an implicit GEMM on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16; the 3-channel first layer 16x16x16): operands
// rounded to nearest-even from FP32 (v_cvt_pk_bf16_f32), FP32 accumulation.
// Forward: one wave per image; backward: two waves per image, each owning
// one 16-channel half of every layer's outputs.  Activations live in LDS
// tiles of 16 x 16 pixels x 32 channels (16 KB), pixel-major or
// channel-major with XOR-swizzled 16-byte chunks; a layer's weights sit in
// registers as matrix-core fragments, staged in BF16 once per call.  A
// pixel's left and right neighbours come from the lanes beside it (DPP row
// shifts, zero past the image's edge), so each row of a tile is read once
// per layer.  Weight gradients are summed over the few images a workgroup
// takes into one partial row per workgroup, and the rows in a fixed order
// afterwards, so every result is deterministic for a given batch size.
#include "cnn_kernels.hpp"

namespace lbm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NC = 32;  // channels of every hidden layer

// FP32 -> BF16, round to nearest even, in hardware: one value, or two packed
// (lo in the low half).
__device__ __forceinline__ unsigned short f2bf(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
__device__ __forceinline__ unsigned pk_bf16(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
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

// The layers' weights as matrix-core fragments in BF16, once per call:
// layer 1 [k-step 3][o tile 2][lane 64][4] (o = 16 tile + lane % 16, tap =
// 4 k-step + lane / 16, channel slot j; slot 3 and taps past 8 zero); layers 2
// and 3 [tap 9][tile 2][lane 64][8], forward with rows = output channels o =
// 16 tile + lane % 16 and k = input channel 8 (lane / 16) + j, then
// transposed for the data gradient (rows = input channels, k = o).
__global__ __launch_bounds__(256) void cnn_stage_weights_kernel(const float* __restrict__ params,
                                                                unsigned short* __restrict__ wt) {
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= CNN_WT_ELEMS) return;
    float v = 0.0f;
    if (e < CNN_FRAG1_ELEMS) {
        const int j = e & 3, lane = (e >> 2) & 63, mt = (e >> 8) & 1, ks = e >> 9;
        const int o = 16 * mt + (lane & 15), tap = 4 * ks + (lane >> 4);
        if (tap < 9 && j < 3) v = params[CNN_OFF_W1 + (o * 3 + j) * 9 + tap];
    } else {
        const int r0 = e - CNN_FRAG2_OFF;
        const int which = r0 / CNN_FRAG23_ELEMS;  // 0, 1: layers 2, 3 forward; 2, 3: transposed
        const int r = r0 - which * CNN_FRAG23_ELEMS;
        const int j = r & 7, lane = (r >> 3) & 63, mt = (r >> 9) & 1, tap = r >> 10;
        const int row = 16 * mt + (lane & 15), kk = 8 * (lane >> 4) + j;
        const int o = which < 2 ? row : kk, c = which < 2 ? kk : row;
        v = params[((which & 1) == 0 ? CNN_OFF_W2 : CNN_OFF_W3) + (o * NC + c) * 9 + tap];
    }
    wt[e] = f2bf(v);
}

// One bf16x8 from 16 bytes of LDS.
__device__ __forceinline__ bf16x8 lds_b8(const unsigned short* p) {
    return __builtin_bit_cast(bf16x8, *(const uint4*)p);
}

// The 16-byte fragment of the lane's neighbour one pixel to the left (SHR) or
// right (SHL) within its row of 16 lanes; zero past the row's ends.
template <int CTRL>
__device__ __forceinline__ bf16x8 dpp_shift(bf16x8 v) {
    uint4 u = __builtin_bit_cast(uint4, v);
    u.x = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u.x, CTRL, 0xf, 0xf, true);
    u.y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u.y, CTRL, 0xf, 0xf, true);
    u.z = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u.z, CTRL, 0xf, 0xf, true);
    u.w = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u.w, CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(bf16x8, u);
}
constexpr int DPP_ROW_SHR1 = 0x111;  // lane i takes lane i - 1 of its row
constexpr int DPP_ROW_SHL1 = 0x101;  // lane i takes lane i + 1 of its row

// (px, ch) in a pixel-major tile: 8-channel chunks swizzled by pixel / 4.
__device__ __forceinline__ int pm_idx(int px, int ch) {
    return px * NC + ((((ch >> 3) ^ (px >> 2)) & 3) << 3) + (ch & 7);
}
// (ch, px) in a channel-major tile: 8-pixel chunks swizzled by channel % 16.
__device__ __forceinline__ int cm_idx(int ch, int px) {
    return ch * 256 + ((((px >> 3) ^ ch) & 31) << 3) + (px & 7);
}

__device__ __forceinline__ unsigned funnel16(unsigned hi, unsigned lo) { return __builtin_amdgcn_alignbit(hi, lo, 16); }

// The eight pixels x0 + dx .. x0 + dx + 7 (x0 = 0 or 8, dx = -1, 0, 1, zero
// outside 0..15) of a row given as h0 = pixels 0..7 and h1 = 8..15.
__device__ __forceinline__ uint4 row_window(uint4 h0, uint4 h1, bool left_half, int dx) {
    const uint4 m = left_half ? h0 : h1;
    if (dx == 0) return m;
    if (dx < 0) {
        const unsigned l = left_half ? 0u : h0.w;
        return uint4{funnel16(m.x, l), funnel16(m.y, m.x), funnel16(m.z, m.y), funnel16(m.w, m.z)};
    }
    const unsigned r = left_half ? h1.x : 0u;
    return uint4{funnel16(m.y, m.x), funnel16(m.z, m.y), funnel16(m.w, m.z), funnel16(r, m.w)};
}

// ---- forward: one wave per image ------------------------------------------

// ReLU and BF16 of the lane's output values of one row (bias already in the
// accumulators; two output tiles: channels 16 mt + 4 (lane / 16) + j of pixel
// lane % 16); into the pixel-major tile (or, for the last layer, the channel
// sums cs instead) and the saved activation, 8 bytes each.
template <bool LAST>
__device__ __forceinline__ void fwd_row_out(const f32x4 acc[2], int y, int col, int g, unsigned short* tile,
                                            unsigned short* __restrict__ act, f32x4 cs[2]) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = fmaxf(acc[mt][j], 0.0f);
        const uint2 o = uint2{pk_bf16(v[0], v[1]), pk_bf16(v[2], v[3])};
        const int c0 = 16 * mt + 4 * g, px = y * 16 + col;
        if (LAST)
            cs[mt] += v;
        else
            *(uint2*)(tile + pm_idx(px, c0)) = o;
        if (act) *(uint2*)(act + px * NC + c0) = o;
    }
}

// One 32 -> 32 layer of the wave's image, in place in its tile, as a sweep
// over the input rows: each input row is read from LDS once (lane: 8 channels
// of one pixel; the next row's read is issued before this row's products),
// its left and right neighbours come from the lanes beside it, and it feeds
// all nine taps, i.e. the output rows above, on and below it.  Output row y
// is complete once input row y + 1 has been swept; it is written one row
// later, over input row y, which no remaining output reads (a wave's LDS
// accesses complete in program order).  Accumulators of four output rows
// rotate, each starting from the bias.  The last layer keeps its outputs out
// of the tile and sums them per channel (cs).
template <bool LAST>
__device__ __forceinline__ void fwd_layer32(unsigned short* tile, const unsigned short* __restrict__ frag,
                                            const float* __restrict__ bias_p, unsigned short* __restrict__ act,
                                            f32x4 cs[2], int lane) {
    const int col = lane & 15, g = lane >> 4;
    bf16x8 w[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
            w[t][mt] = __builtin_bit_cast(bf16x8, *(const uint4*)(frag + ((t * 2 + mt) * 64 + lane) * 8));
    f32x4 b0[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) b0[mt][j] = bias_p[16 * mt + 4 * g + j];
    f32x4 acc[4][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) acc[0][mt] = b0[mt];
    bf16x8 next = lds_b8(tile + pm_idx(col, 8 * g));
#pragma unroll
    for (int ys = 0; ys < 16; ++ys) {
        const bf16x8 v0 = next;
        if (ys < 15) next = lds_b8(tile + pm_idx((ys + 1) * 16 + col, 8 * g));
        const bf16x8 vm = dpp_shift<DPP_ROW_SHR1>(v0), vp = dpp_shift<DPP_ROW_SHL1>(v0);  // pixels x - 1, x + 1
        if (ys < 15) {
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) acc[(ys + 1) & 3][mt] = b0[mt];
        }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {  // output row ys + 1 - dy reads this row through tap (dy, dx)
                const int y = ys + 1 - dy;
                if (y < 0 || y > 15) continue;
                const bf16x8 v = dx == 0 ? vm : (dx == 1 ? v0 : vp);
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) acc[y & 3][mt] = mfma32(w[dy * 3 + dx][mt], v, acc[y & 3][mt]);
            }
        if (ys >= 2) fwd_row_out<LAST>(acc[(ys - 2) & 3], ys - 2, col, g, tile, act, cs);
    }
    fwd_row_out<LAST>(acc[14 & 3], 14, col, g, tile, act, cs);
    fwd_row_out<LAST>(acc[15 & 3], 15, col, g, tile, act, cs);
}

__global__ __launch_bounds__(64) void cnn_forward_kernel(CnnArgs a) {
    __shared__ uint4 tile4[256 * NC / 8];  // the activation tile, pixel-major
    __shared__ uint2 in2[256];             // the input picture: 16 x 16 pixels x 4 channel slots
    __shared__ float gs[NC];
    unsigned short* const tile = (unsigned short*)tile4;
    const int b = (int)blockIdx.x;
    const int lane = (int)threadIdx.x, col = lane & 15, g = lane >> 4;
    const float* p = a.params;
    unsigned short* const act = a.act ? a.act + (long long)b * 3 * 256 * NC : nullptr;
    // the picture in BF16, pixel-major, channel slot 3 zero
    const float* x = a.x + (long long)b * 3 * 256;
    for (int q = lane; q < 256; q += 64) in2[q] = uint2{pk_bf16(x[q], x[256 + q]), pk_bf16(x[512 + q], 0.0f)};
    __syncthreads();
    // layer 1 (3 -> 32): k = (tap, channel slot), tap = 4 k-step + lane / 16
    {
        const unsigned short* f1 = a.wt + CNN_FRAG1_OFF;
        bf16x4 w1[3][2];
#pragma unroll
        for (int ks = 0; ks < 3; ++ks)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
                w1[ks][mt] = __builtin_bit_cast(bf16x4, *(const uint2*)(f1 + ((ks * 2 + mt) * 64 + lane) * 4));
        f32x4 b0[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) b0[mt][j] = p[CNN_OFF_B1 + 16 * mt + 4 * g + j];
        for (int y0 = 0; y0 < 16; y0 += 2) {
            f32x4 cur[2][2];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) cur[r][mt] = b0[mt];
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
            fwd_row_out<false>(cur[0], y0, col, g, tile, act, nullptr);
            fwd_row_out<false>(cur[1], y0 + 1, col, g, tile, act, nullptr);
        }
    }
    __syncthreads();
    fwd_layer32<false>(tile, a.wt + CNN_FRAG2_OFF, p + CNN_OFF_B2, act ? act + 256 * NC : nullptr, nullptr, lane);
    __syncthreads();
    f32x4 cs[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
    fwd_layer32<true>(tile, a.wt + CNN_FRAG3_OFF, p + CNN_OFF_B3, act ? act + 2 * 256 * NC : nullptr, cs, lane);
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

// ---- backward: two waves per image ----------------------------------------
//
// LDS of the image: two 16 KB tiles of 256 pixels x 32 channels (BF16)
// (32 KB: five images per compute unit).  A tile is channel-major (rows of
// 256 pixels) or pixel-major (32 channels per pixel); it changes between the
// two in place, by 8 x 8 block transposes in registers.  Wave w owns output
// tile w (16 channels) of every GEMM below.  Weight gradient of a layer, per
// tap, dW[o][c] = sum_p dZ[p][o] X[p + d][c] with K = pixels: A = dZ^T chunks,
// B = X chunks shifted by the tap, both channel-major, B built in registers
// from two aligned 16-byte reads of the row (a shift by one pixel is a 16-bit
// funnel shift); all nine taps at once, so that each A chunk is read once.
// Data gradient, dX[q][c] = sum_{tap, o} dZ[q - d][o] W[o][c][tap] with K =
// output channels: A = pixel-major dZ rows (a sweep as in the forward), B = the
// transposed weight fragments in registers; each lane's result is four
// neighbouring pixels of one channel, so the ReLU mask of the layer below
// (its saved activation, the X tile) is read and dZ of that layer written over
// it in 8-byte pieces, channel-major, ready for the next weight gradient.

// 8 x 8 transpose of 16-bit elements: out[j] element i = in[i] element j.
__device__ __forceinline__ void tr8x8(const uint4 in[8], uint4 out[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 lo = in[2 * q], hi = in[2 * q + 1];
            const unsigned a = (j >> 1) == 0 ? lo.x : (j >> 1) == 1 ? lo.y : (j >> 1) == 2 ? lo.z : lo.w;
            const unsigned c = (j >> 1) == 0 ? hi.x : (j >> 1) == 1 ? hi.y : (j >> 1) == 2 ? hi.z : hi.w;
            w[q] = (j & 1) ? ((a >> 16) | (c & 0xffff0000u)) : ((a & 0xffffu) | (c << 16));
        }
        out[j] = uint4{w[0], w[1], w[2], w[3]};
    }
}

// The 8 x 8 blocks of a tile: 32 pixel chunks x 4 channel chunks, one per
// thread of the image's workgroup: pixels 8 kp .. 8 kp + 7 and channels
// 8 c8 .. 8 c8 + 7 with c8 = tid % 4 and kp = tid / 4.

// A saved activation (pixel-major [256][32] in global memory) into a
// channel-major tile.
__device__ void stage_cm(const unsigned short* __restrict__ act, unsigned short* xc, int tid) {
    const int c8 = tid & 3, kp = tid >> 2;
    uint4 v[8], t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = *(const uint4*)(act + (8 * kp + q) * NC + 8 * c8);
    tr8x8(v, t);
#pragma unroll
    for (int j = 0; j < 8; ++j) *(uint4*)(xc + cm_idx(8 * c8 + j, 8 * kp)) = t[j];
}

// A channel-major tile made pixel-major, in place (every read before the
// first write).
__device__ void cm_to_pm(unsigned short* t, int tid) {
    const int c8 = tid & 3, kp = tid >> 2;
    uint4 v[8], o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = *(const uint4*)(t + cm_idx(8 * c8 + j, 8 * kp));
    __syncthreads();
    tr8x8(v, o);
#pragma unroll
    for (int q = 0; q < 8; ++q) *(uint4*)(t + pm_idx(8 * kp + q, 8 * c8)) = o[q];
}

// Weight gradient of a 32 -> 32 layer, the wave's input-channel tile nt:
// all nine taps (3 x 3 x 2 accumulator tiles), added to out (the partial
// layout: per tap and tile, each lane's four values), which the first image
// of a workgroup (first) writes instead.
__device__ void bwd_wgrad32(const unsigned short* dzc, const unsigned short* xc, float* __restrict__ out, bool first,
                            int lane, int nt) {
    const int col = lane & 15, g = lane >> 4;
    const bool left = (g & 1) == 0;
    const int c = 16 * nt + col;
    __asm__ volatile("" ::: "memory");  // the partial loads below stay here
    f32x4 acc[3][3][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            // loaded either way (workspace memory; a branch per load would split the code)
            const f32x4 v = *(const f32x4*)(out + (((t * 2 + mt) * 2 + nt) * 64 + lane) * 4);
            acc[t / 3][t % 3][mt] = first ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : v;
        }
#pragma unroll 2
    for (int ks = 0; ks < 8; ++ks) {
        bf16x8 av[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) av[mt] = lds_b8(dzc + cm_idx(16 * mt + col, 32 * ks + 8 * g));
        const int y = 2 * ks + (g >> 1);  // the lane's K row
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yr = y + dy - 1;
            const bool rok = yr >= 0 && yr < 16;
            const int yc = rok ? yr : 0;
            uint4 h0 = *(const uint4*)(xc + cm_idx(c, yc * 16));
            uint4 h1 = *(const uint4*)(xc + cm_idx(c, yc * 16 + 8));
            if (!rok) h0 = h1 = uint4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const bf16x8 bv = __builtin_bit_cast(bf16x8, row_window(h0, h1, left, dx - 1));
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) acc[dy][dx][mt] = mfma32(av[mt], bv, acc[dy][dx][mt]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) *(f32x4*)(out + (((t * 2 + mt) * 2 + nt) * 64 + lane) * 4) = acc[t / 3][t % 3][mt];
}

// Weight gradient of the first layer (3 input channels), the wave's column
// tile nt: columns n = 3 tap + c (27 of 32, the others zero), each lane's
// column with its own tap; added to out in the partial layout (written by
// the first image).
__device__ void bwd_wgrad1(const unsigned short* dzc, const unsigned short* xc, float* __restrict__ out, bool first,
                           int lane, int nt) {
    const int col = lane & 15, g = lane >> 4;
    const bool left = (g & 1) == 0;
    const int n = 16 * nt + col;
    const int tap = n / 3, c = n - 3 * (n / 3);
    const int dy = tap / 3 - 1, dx = tap - 3 * (tap / 3) - 1;
    __asm__ volatile("" ::: "memory");  // the partial loads below stay here
    f32x4 acc[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const f32x4 v = *(const f32x4*)(out + ((mt * 2 + nt) * 64 + lane) * 4);
        acc[mt] = first ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : v;
    }
    for (int ks = 0; ks < 8; ++ks) {
        bf16x8 av[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) av[mt] = lds_b8(dzc + cm_idx(16 * mt + col, 32 * ks + 8 * g));
        const int y = 2 * ks + (g >> 1);
        const int yr = y + dy;
        const bool rok = n < 27 && yr >= 0 && yr < 16;
        const int yc = rok ? yr : y, cc = n < 27 ? c : 0;
        uint4 h0 = *(const uint4*)(xc + cm_idx(cc, yc * 16));
        uint4 h1 = *(const uint4*)(xc + cm_idx(cc, yc * 16 + 8));
        if (!rok) h0 = h1 = uint4{0u, 0u, 0u, 0u};
        const uint4 wm = row_window(h0, h1, left, -1), w0 = row_window(h0, h1, left, 0),
                    wp = row_window(h0, h1, left, 1);
        const bf16x8 bv = __builtin_bit_cast(bf16x8, dx < 0 ? wm : (dx == 0 ? w0 : wp));
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[mt] = mfma32(av[mt], bv, acc[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) *(f32x4*)(out + ((mt * 2 + nt) * 64 + lane) * 4) = acc[mt];
}

// One row of a data gradient's output: lane (col, g) holds dX of channel
// 16 nt + col at pixels 4 g .. 4 g + 3 of row y.  dZ of the layer below =
// [a > 0] dX (a: that layer's activation, held channel-major in xz) replaces
// a in xz; bs sums it.
__device__ __forceinline__ void bwd_row_out(f32x4 acc, unsigned short* xz, int y, int col, int g, int nt,
                                            float& bs) {
    uint2* const q = (uint2*)(xz + cm_idx(16 * nt + col, y * 16 + 4 * g));
    const uint2 m = *q;
    const unsigned short mb[4] = {(unsigned short)m.x, (unsigned short)(m.x >> 16), (unsigned short)m.y,
                                  (unsigned short)(m.y >> 16)};
    float d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        d[j] = bf2f(mb[j]) > 0.0f ? acc[j] : 0.0f;
        bs += d[j];
    }
    *q = uint2{pk_bf16(d[0], d[1]), pk_bf16(d[2], d[3])};
    // the row's sum taken now: left to the scheduler, the additions sink to
    // the end of the sweep and every row's d stays live in registers
    __asm__ volatile("" : "+v"(bs));
}

// Data gradient of a 32 -> 32 layer, the wave's output-channel tile nt, from
// dZ (pixel-major, dzp) into xz (the activation of the layer below,
// channel-major: its mask, replaced by its dZ): a sweep over the rows of dZ as
// in the forward, each row read once and shifted a pixel either way between
// lanes, feeding the output rows above, on and below it; output row y is
// written once dZ row y + 2 has been swept.
__device__ void bwd_dgrad32(const unsigned short* dzp, unsigned short* xz, const unsigned short* __restrict__ ft,
                            float& bs, int lane, int nt) {
    const int col = lane & 15, g = lane >> 4;
    bf16x8 w[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) w[t] = __builtin_bit_cast(bf16x8, *(const uint4*)(ft + ((t * 2 + nt) * 64 + lane) * 8));
    f32x4 acc[4];
    acc[0] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 next = lds_b8(dzp + pm_idx(col, 8 * g));
#pragma unroll
    for (int ys = 0; ys < 16; ++ys) {
        const bf16x8 v0 = next;
        if (ys < 15) next = lds_b8(dzp + pm_idx((ys + 1) * 16 + col, 8 * g));
        // output pixel x reads dZ pixel x - dx: dx = -1, 0, 1
        const bf16x8 vl = dpp_shift<DPP_ROW_SHL1>(v0), vr = dpp_shift<DPP_ROW_SHR1>(v0);  // pixels x + 1, x - 1
        if (ys < 15) acc[(ys + 1) & 3] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {  // output row ys + dy - 1 reads this row through tap (dy, dx)
                const int y = ys + dy - 1;
                if (y < 0 || y > 15) continue;
                const bf16x8 v = dx == 0 ? vl : (dx == 1 ? v0 : vr);
                acc[y & 3] = mfma32(v, w[dy * 3 + dx], acc[y & 3]);
            }
        if (ys >= 2) bwd_row_out(acc[(ys - 2) & 3], xz, ys - 2, col, g, nt, bs);
    }
    bwd_row_out(acc[14 & 3], xz, 14, col, g, nt, bs);
    bwd_row_out(acc[15 & 3], xz, 15, col, g, nt, bs);
}

// Per-channel total of bs (channel 16 nt + lane % 16) over the four lanes of
// the channel, in a fixed order, into out[channel].
__device__ __forceinline__ void bsum_out(float bs, float* __restrict__ out, int lane, int nt) {
    bs += __shfl_xor(bs, 16, 64);
    bs += __shfl_xor(bs, 32, 64);
    if (lane < 16) out[16 * nt + lane] = bs;
}

// Backward of the images ipw k .. ipw k + ipw - 1 (workgroup k) given their
// saved activations, one after the other; their parameter gradients are
// summed into partial row k (each lane adds into its own pieces of the row,
// which stays in the caches between images).
__global__ __launch_bounds__(128, 2) void cnn_backward_kernel(CnnArgs a) {
    __shared__ uint4 tile_p[256 * NC / 8];
    __shared__ uint4 tile_q[256 * NC / 8];
    __shared__ float bred[2][NC];
    unsigned short* const P = (unsigned short*)tile_p;
    unsigned short* const Q = (unsigned short*)tile_q;
    const float* p = a.params;
    const int ipw = cnn_images_per_group(a.batch);
    const int b0 = (int)blockIdx.x * ipw, b1 = min(b0 + ipw, a.batch);
    float* const part = a.partial + (long long)blockIdx.x * CNN_PART_STRIDE;
    const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6, c8 = tid & 3;
    float bs8[8], bs2 = 0.0f, bs1 = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) bs8[j] = 0.0f;
    for (int b = b0; b < b1; ++b) {
        // the thread index laundered once per image: every LDS address and
        // weight load derived from it is then computed where it is used, not
        // hoisted out of the loop to hold registers through every image
        int tid = (int)threadIdx.x;
        __asm__ volatile("" : "+v"(tid) :: "memory");
        const int lane = tid & 63, wv = tid >> 6;
        const int c8 = tid & 3, kp = tid >> 2;  // the thread's 8 x 8 block of a tile
        const unsigned short* act = a.act + (long long)b * 3 * 256 * NC;  // a1, a2, a3
        // dL/dy for the mean squared error, then through the read-out and the average
        const float gy = 2.0f * (a.y[b] - a.labels[b]) / (float)a.batch;
        // ---- layer 3: dZ3 = [a3 > 0] dG, dG = gy w4 / 256, channel-major into
        // Q; a2 (the input of layer 3) channel-major into P
        {
            const unsigned short* a3 = act + 2 * 256 * NC;
            uint4 va[8], vx[8];  // every load in flight before the first is used
#pragma unroll
            for (int q = 0; q < 8; ++q) va[q] = *(const uint4*)(a3 + (8 * kp + q) * NC + 8 * c8);
#pragma unroll
            for (int q = 0; q < 8; ++q) vx[q] = *(const uint4*)(act + 256 * NC + (8 * kp + q) * NC + 8 * c8);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float dg = gy * p[CNN_OFF_W4 + 8 * c8 + j] * (1.0f / 256.0f);
                float d[8];
                int n = 0;  // pixels where channel j is active: its bias gradient is n dg
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint4 v = va[q];
                    const unsigned w = (j >> 1) == 0 ? v.x : (j >> 1) == 1 ? v.y : (j >> 1) == 2 ? v.z : v.w;
                    const bool on = bf2f((unsigned short)(w >> (16 * (j & 1)))) > 0.0f;
                    d[q] = on ? dg : 0.0f;
                    n += on;
                }
                bs8[j] += (float)n * dg;
                *(uint4*)(Q + cm_idx(8 * c8 + j, 8 * kp)) =
                    uint4{pk_bf16(d[0], d[1]), pk_bf16(d[2], d[3]), pk_bf16(d[4], d[5]), pk_bf16(d[6], d[7])};
            }
            uint4 t[8];
            tr8x8(vx, t);
#pragma unroll
            for (int j = 0; j < 8; ++j) *(uint4*)(P + cm_idx(8 * c8 + j, 8 * kp)) = t[j];
        }
        __syncthreads();
        bwd_wgrad32(Q, P, part + CNN_PART_W3, b == b0, lane, wv);
        __syncthreads();
        cm_to_pm(Q, tid);
        __syncthreads();
        bwd_dgrad32(Q, P, a.wt + CNN_FRAGT3_OFF, bs2, lane, wv);  // P: a2 -> dZ2
        __syncthreads();
        stage_cm(act, Q, tid);  // a1, the input of layer 2
        __syncthreads();
        bwd_wgrad32(P, Q, part + CNN_PART_W2, b == b0, lane, wv);
        __syncthreads();
        cm_to_pm(P, tid);
        __syncthreads();
        bwd_dgrad32(P, Q, a.wt + CNN_FRAGT2_OFF, bs1, lane, wv);  // Q: a1 -> dZ1
        __syncthreads();
        // the picture in BF16, channel-major (rows 0..2 of P)
        const float* x = a.x + (long long)b * 3 * 256;
        for (int q = tid; q < 3 * 256; q += 128) P[cm_idx(q >> 8, q & 255)] = f2bf(x[q]);
        __syncthreads();
        bwd_wgrad1(Q, P, part + CNN_PART_W1, b == b0, lane, wv);
        __syncthreads();  // the next image overwrites both tiles
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float v = bs8[j];
#pragma unroll
        for (int m = 4; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
        if (lane < 4) bred[wv][8 * c8 + j] = v;
    }
    bsum_out(bs2, part + CNN_PART_B2, lane, wv);
    bsum_out(bs1, part + CNN_PART_B1, lane, wv);
    __syncthreads();
    if (tid < NC) {
        part[CNN_PART_B3 + tid] = bred[0][tid] + bred[1][tid];
        float s = 0.0f;  // the read-out: sum over the images of gy times the averages
        for (int b = b0; b < b1; ++b) s += 2.0f * (a.y[b] - a.labels[b]) / (float)a.batch * a.gap[(long long)b * NC + tid];
        part[CNN_PART_W4 + tid] = s;
    } else if (tid == NC) {
        float s = 0.0f;
        for (int b = b0; b < b1; ++b) s += 2.0f * (a.y[b] - a.labels[b]) / (float)a.batch;
        part[CNN_PART_B4] = s;
    } else if (tid < NC + 4) {
        part[CNN_PART_B4 + tid - NC] = 0.0f;  // the row's three unused columns
    }
}

// Gradients summed over the partial rows (one per backward workgroup) in a
// fixed order, in two passes: pass 1 sums each chunk of rows in row order
// into the chunk's first row, pass 2 sums those rows in chunk order and, in
// its first workgroup, the loss (a fixed-order tree).  Deterministic for a
// given batch size.  Chunks hold about sqrt(rows) rows (a power of two, 8 to
// 256), so that neither pass runs a long chain of dependent loads.
__host__ __device__ inline int red_chunk(int rows) {
    int c = 8;
    while (c < 256 && c * c < rows) c *= 2;
    return c;
}

__global__ __launch_bounds__(256) void cnn_reduce_chunks_kernel(CnnArgs a) {
    const int r4 = 4 * (int)(blockIdx.x * blockDim.x + threadIdx.x);  // four columns
    if (r4 >= CNN_PART) return;
    const int rows = cnn_partial_rows(a.batch);
    const int rc = red_chunk(rows);
    const int k0 = (int)blockIdx.y * rc, k1 = min(k0 + rc, rows);
    float4 tot = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float* src = a.partial + (long long)k0 * CNN_PART_STRIDE + r4;
#pragma unroll 8
    for (int k = k0; k < k1; ++k, src += CNN_PART_STRIDE) {
        const float4 v = *(const float4*)src;
        tot.x += v.x;
        tot.y += v.y;
        tot.z += v.z;
        tot.w += v.w;
    }
    *(float4*)(a.partial + (long long)k0 * CNN_PART_STRIDE + r4) = tot;  // the chunk's first row, read only by this thread
}

// The parameter (canonical order) held in column r of a partial row, or -1.
__device__ __forceinline__ int canon_index(int r) {
    if (r >= CNN_PART) return -1;
    if (r == CNN_PART_B4) return CNN_OFF_B4;
    if (r >= CNN_PART_W4) return CNN_OFF_W4 + (r - CNN_PART_W4);
    if (r >= CNN_PART_B1) return CNN_OFF_B1 + (r - CNN_PART_B1);
    if (r >= CNN_PART_B2) return CNN_OFF_B2 + (r - CNN_PART_B2);
    if (r >= CNN_PART_B3) return CNN_OFF_B3 + (r - CNN_PART_B3);
    if (r >= CNN_PART_W1) {  // [o tile][n tile][lane][j], column n = 3 tap + c
        const int e = r - CNN_PART_W1, j = e & 3, lane = (e >> 2) & 63, nt = (e >> 8) & 1, mt = e >> 9;
        const int o = 16 * mt + 4 * (lane >> 4) + j, n = 16 * nt + (lane & 15);
        if (n >= 27) return -1;
        return CNN_OFF_W1 + (o * 3 + n % 3) * 9 + n / 3;
    }
    const bool l2 = r >= CNN_PART_W2;  // [tap][o tile][c tile][lane][j]
    const int e = r - (l2 ? CNN_PART_W2 : CNN_PART_W3), j = e & 3, lane = (e >> 2) & 63;
    const int nt = (e >> 8) & 1, mt = (e >> 9) & 1, t = e >> 10;
    const int o = 16 * mt + 4 * (lane >> 4) + j, c = 16 * nt + (lane & 15);
    return (l2 ? CNN_OFF_W2 : CNN_OFF_W3) + (o * NC + c) * 9 + t;
}

__global__ __launch_bounds__(256) void cnn_reduce_final_kernel(CnnArgs a) {
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);  // a partial column
    const int rows = cnn_partial_rows(a.batch);
    const int rc = red_chunk(rows);
    const int chunks = (rows + rc - 1) / rc;
    const int dst = canon_index(r);
    if (dst >= 0) {
        float tot = 0.0f;
        const float* src = a.partial + r;
#pragma unroll 8
        for (int c = 0; c < chunks; ++c, src += (long long)rc * CNN_PART_STRIDE) tot += *src;  // loads in flight, sums in order
        a.grads[dst] = tot;
    }
    if (blockIdx.x == 0 && a.loss) {  // the whole first workgroup
        __shared__ double red[256];
        double l = 0.0;
        for (int b = (int)threadIdx.x; b < a.batch; b += 256) {
            const double d = (double)a.y[b] - (double)a.labels[b];
            l += d * d;
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
    const int mi = a.list ? a.list[blockIdx.x] : a.m0 + (int)blockIdx.x;
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
    const int rows = cnn_partial_rows(a.batch);
    hipLaunchKernelGGL(cnn_backward_kernel, dim3(rows), dim3(128), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned chunks = (unsigned)((rows + red_chunk(rows) - 1) / red_chunk(rows));
    hipLaunchKernelGGL(cnn_reduce_chunks_kernel, dim3((CNN_PART + 1023) / 1024, chunks), dim3(256), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(cnn_reduce_final_kernel, dim3((CNN_PART + 255) / 256), dim3(256), 0, st, a);
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
