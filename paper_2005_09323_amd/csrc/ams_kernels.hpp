// Argument block of the AMS selection kernels.
#pragma once

#include "common.hpp"

namespace lbm {

constexpr int MAX_AMS = 2048;  // members one selection workgroup handles (LDS-resident)

struct AmsArgs {
    const float* series;  // [n][t_len]
    int n;
    int t_len;
    int n_kill;
    int iteration;
    uint64_t key;
    float* maxima;   // [n] out
    int* killed;     // [n] out, first n_killed valid
    int* parent;     // [n] out
    int* branch_t;   // [n] out
    int* n_killed;   // [1] out
    float* level;    // [1] out
};

hipError_t launch_ams(const AmsArgs& a, hipStream_t st);

}  // namespace lbm
