// Argument blocks of the score-network and feature kernels.
#pragma once

#include "common.hpp"

namespace lbm {

// Parameter vector (FP32), in the order w1[32][3][3][3], b1[32], w2[32][32][3][3],
// b2[32], w3[32][32][3][3], b3[32], w4[32], b4.
constexpr int CNN_OFF_W1 = 0, CNN_OFF_B1 = 864, CNN_OFF_W2 = 896, CNN_OFF_B2 = 10112;
constexpr int CNN_OFF_W3 = 10144, CNN_OFF_B3 = 19360, CNN_OFF_W4 = 19392, CNN_OFF_B4 = 19424;
constexpr int CNN_N_PARAMS = 19425;

struct CnnArgs {
    const float* params;
    const float* x;       // [batch][3][16][16]
    const float* labels;  // [batch]
    int batch;
    float* y;             // [batch]
    float* gap;           // [batch][32] averages (saved for the read-out gradient)
    unsigned short* act;  // [batch][3][256][32] BF16 activations (saved for backward)
    float* partial;       // [batch][CNN_N_PARAMS]
    float* grads;         // [CNN_N_PARAMS]
    float* loss;          // [1] or null
    unsigned short* wt;   // BF16 weight tables [layer][kp][32], kp = 32, 288, 288, then the A fragments (staged once per call)
};

constexpr int CNN_TAB_ELEMS = (32 + 288 + 288) * 32;  // the three staged weight tables [k][o]
// The weights again as matrix-core A fragments, one 16-byte (8 x BF16) or
// 8-byte (layer 1) piece per lane: layer 1 [k-step 3][o tile 2][lane 64][4],
// layers 2 and 3 [tap 9][o tile 2][lane 64][8].
constexpr int CNN_FRAG1_ELEMS = 3 * 2 * 64 * 4;
constexpr int CNN_FRAG23_ELEMS = 9 * 2 * 64 * 8;
constexpr int CNN_FRAG_OFF = CNN_TAB_ELEMS;
constexpr int CNN_WT_ELEMS = CNN_TAB_ELEMS + CNN_FRAG1_ELEMS + 2 * CNN_FRAG23_ELEMS;  // everything staged per call

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
    int px0, py0, patch, pool;
    double u_scale, rho_scale;
    float* out;  // [n][3][patch/pool][patch/pool]
};

hipError_t launch_cnn_forward(const CnnArgs& a, hipStream_t st);
hipError_t launch_cnn_backward(const CnnArgs& a, hipStream_t st);
hipError_t launch_cnn_adam(const AdamArgs& a, hipStream_t st);
hipError_t launch_features(const FeatureArgs& a, int n, hipStream_t st);

}  // namespace lbm
