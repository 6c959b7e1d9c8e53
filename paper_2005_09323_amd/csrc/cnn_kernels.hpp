// Argument blocks of the score-network and feature kernels.
#pragma once

#include "common.hpp"

namespace lbm {

// Parameter vector (FP32), in the order w1[32][3][3][3], b1[32], w2[32][32][3][3],
// b2[32], w3[32][32][3][3], b3[32], w4[32], b4.
constexpr int CNN_OFF_W1 = 0, CNN_OFF_B1 = 864, CNN_OFF_W2 = 896, CNN_OFF_B2 = 10112;
constexpr int CNN_OFF_W3 = 10144, CNN_OFF_B3 = 19360, CNN_OFF_W4 = 19392, CNN_OFF_B4 = 19424;
constexpr int CNN_N_PARAMS = 19425;

// Per-image gradient partials, in the order the backward kernel produces
// them (each store a coalesced row of 16-byte pieces): the weight gradients
// of layers 3 and 2 as [tap 9][o tile 2][c tile 2][lane 64][4] (lane l, piece
// j: o = 16 o_tile + 4 (l / 16) + j, c = 16 c_tile + l % 16), of layer 1 as
// [o tile 2][n tile 2][lane 64][4] (column n = 3 tap + c, 27 of 32 used), then
// the biases b3, b2, b1 and the read-out w4, b4.
constexpr int CNN_PART_W3 = 0, CNN_PART_W2 = 9216, CNN_PART_W1 = 18432;
constexpr int CNN_PART_B3 = 19456, CNN_PART_B2 = 19488, CNN_PART_B1 = 19520;
constexpr int CNN_PART_W4 = 19552, CNN_PART_B4 = 19584;
constexpr int CNN_PART = 19585;
constexpr int CNN_PART_STRIDE = 19712;  // floats per partial row (1 KB multiple)

// Images one backward workgroup takes in turn, summing their weight
// gradients in registers into one partial row: up to 8, so that a large
// batch still runs about 2048 workgroups.  Depends on the batch size only.
__host__ __device__ constexpr int cnn_images_per_group(int batch) {
    return batch / 2048 < 1 ? 1 : (batch / 2048 > 8 ? 8 : batch / 2048);
}
__host__ __device__ constexpr int cnn_partial_rows(int batch) {
    return (batch + cnn_images_per_group(batch) - 1) / cnn_images_per_group(batch);
}
// The most rows any batch up to `batch` uses (cnn_partial_rows itself drops
// where the group size steps up, 4095 -> 2048 at 4096): at most 4095 below a
// batch of 16384 (one image per group up to 4095, then groups of k up to
// 2048 (k + 1) - 1 images), ceil(batch / 8) above; the workspace is sized by
// it so that one serves every smaller batch.
__host__ __device__ constexpr int cnn_partial_rows_cap(int batch) {
    return (batch < 4095 ? batch : 4095) > (batch + 7) / 8 ? (batch < 4095 ? batch : 4095) : (batch + 7) / 8;
}

struct CnnArgs {
    const float* params;
    const float* x;       // [batch][3][16][16]
    const float* labels;  // [batch]
    int batch;
    float* y;             // [batch]
    float* gap;           // [batch][32] averages (saved for the read-out gradient)
    unsigned short* act;  // [batch][3][256][32] BF16 activations (saved for backward)
    float* partial;       // [cnn_partial_rows(batch)][CNN_PART_STRIDE]
    float* grads;         // [CNN_N_PARAMS]
    float* loss;          // [1] or null
    unsigned short* wt;   // BF16 weight fragments (staged once per call)
};

// The weights as matrix-core fragments (BF16), staged once per call: layer 1
// as A fragments [k-step 3][o tile 2][lane 64][4], layers 2 and 3 as A
// fragments [tap 9][o tile 2][lane 64][8] (forward: rows = output channels),
// then layers 2 and 3 transposed [tap 9][c tile 2][lane 64][8] (data
// gradient: B fragments with columns = input channels).
constexpr int CNN_FRAG1_ELEMS = 3 * 2 * 64 * 4;
constexpr int CNN_FRAG23_ELEMS = 9 * 2 * 64 * 8;
constexpr int CNN_FRAG1_OFF = 0;
constexpr int CNN_FRAG2_OFF = CNN_FRAG1_OFF + CNN_FRAG1_ELEMS;
constexpr int CNN_FRAG3_OFF = CNN_FRAG2_OFF + CNN_FRAG23_ELEMS;
constexpr int CNN_FRAGT2_OFF = CNN_FRAG3_OFF + CNN_FRAG23_ELEMS;
constexpr int CNN_FRAGT3_OFF = CNN_FRAGT2_OFF + CNN_FRAG23_ELEMS;
constexpr int CNN_WT_ELEMS = CNN_FRAGT3_OFF + CNN_FRAG23_ELEMS;  // everything staged per call

struct AdamArgs {
    float* params;
    float* m;
    float* v;
    const float* grads;
    int step;
    double lr, beta1, beta2, eps;
};

struct FeatureArgs {
    const MemberDev* members;
    const int* parity;
    const float* pop0;
    const float* pop1;
    int m0;
    const int* list;  // member of output row b: list[b], or m0 + b where null
    int px0, py0, patch, pool;
    double u_scale, rho_scale;
    float* out;  // [n][3][patch/pool][patch/pool]
};

hipError_t launch_cnn_forward(const CnnArgs& a, hipStream_t st);
hipError_t launch_cnn_backward(const CnnArgs& a, hipStream_t st);
hipError_t launch_cnn_adam(const AdamArgs& a, hipStream_t st);
hipError_t launch_features(const FeatureArgs& a, int n, hipStream_t st);

}  // namespace lbm
