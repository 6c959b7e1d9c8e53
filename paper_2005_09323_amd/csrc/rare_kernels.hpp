// Argument blocks of the GKTL / perturbation / AMS kernels.
#pragma once

#include "common.hpp"

namespace lbm {

constexpr int MAX_SELECT = 4096;  // members a selection workgroup handles
constexpr int MAX_SNAP = 16;      // perturbation snapshots
constexpr int MASS_CHUNK = 1 << 16;  // floats per mass partial

enum { MODE_SKIP = 0, MODE_COPY = 1, MODE_PERTURB = 2 };

struct MaskWords {
    unsigned w[MAX_SELECT / 32];
};

struct SelectArgs {
    const MemberDev* members;  // current blocks (off) of the states
    const int* parity;         // current parities
    int relabel;        // 1: place copies by relabelling blocks (tables below), 0: gather every copy
    long long* new_off; // [n] out (relabel): the block each slot's state occupies after the clone
    int* new_parity;    // [n] out (relabel): its buffer
    int* extra;         // [n] out (relabel): slots whose state is written (copies beyond the first), in order
    int* n_extra;       // [1] out (relabel)
    const double* accum;
    double k;
    uint64_t key;
    int period;
    int n;
    int n_snap;
    double eps;
    double* prefix;     // [n] scratch
    double* ln_r;       // [1] out
    int* ancestors;     // [n] out
    int* status;        // [1] out: 1 if every weight is non-finite
    int* mode;          // [n]
    int* src;           // [n]
    int* need_mass;     // [n]
    double* alpha;      // [n][MAX_SNAP]
    double* alpha_sum;  // [n]
};

struct PlanArgs {
    MaskWords mask;
    uint64_t key;
    int period;
    int n;
    int n_snap;
    int* mode;
    int* src;
    int* need_mass;
    double* alpha;
    double* alpha_sum;
};

struct MassArgs {
    const MemberDev* members;
    const int* parity;
    const int* need_mass;
    const float* pop0;
    const float* pop1;
    const float* snapshots;  // [n_snap][9][ny][nx]
    double* partial;         // [(n + n_snap) * blocks_per_state]
    int n;
    int blocks_per_state;
};

struct ScaleArgs {
    const int* mode;
    const int* src;
    const double* partial;
    const double* alpha;
    const double* alpha_sum;
    double* scale;
    double* coef_w;
    double n_fluid;
    double eps;
    int n;
    int n_snap;
    int blocks_per_state;
};

struct GatherArgs {
    const MemberDev* members;
    const int* parity;
    const int* mode;
    const int* src;
    float* pop0;  // read (source state) and written (new state): never the same member block
    float* pop1;
    const float* snapshots;
    const double* alpha;
    const double* scale;
    const double* coef_w;
    double eps;
    int n;
    int n_snap;
};

// Relabelling clone: the copies beyond the first of each ancestor, written
// into the blocks of states that left no descendant (same buffer as the
// ancestor); the first copy of each ancestor keeps the ancestor's block.
struct PlaceArgs {
    const MemberDev* members;  // blocks before the clone (the ancestors' states)
    const int* parity;         // parities before the clone
    const int* extra;          // [n_extra] slots to write
    const int* src;            // [n] ancestor of each slot
    const int* mode;           // [n] MODE_COPY or MODE_PERTURB
    const long long* new_off;  // [n] destination block of each slot
    float* pop0;
    float* pop1;
    const float* snapshots;
    const double* alpha;
    const double* scale;
    const double* coef_w;
    double eps;
    int n_snap;
    int n_extra;  // entries of extra
};

struct CommitArgs {
    MemberDev* members;
    int* parity;
    const long long* new_off;
    const int* new_parity;
    double* accum;
    int* flags;
    const int* flags_new;
    int n;
};

struct FinishArgs {
    const int* mode;
    const int* src;
    int* parity;
    double* accum;
    int* flags;
    int* flags_new;
    int n;
    int reset_accum;
};

hipError_t launch_select(const SelectArgs& a, hipStream_t st);
hipError_t launch_plan(const PlanArgs& a, hipStream_t st);
hipError_t launch_mass(const MassArgs& a, int n_states, hipStream_t st);
hipError_t launch_scale(const ScaleArgs& a, hipStream_t st);
hipError_t launch_gather(const GatherArgs& a, long long floats_per_member, hipStream_t st);
hipError_t launch_finish(const FinishArgs& a, hipStream_t st);
hipError_t launch_place(const PlaceArgs& a, long long floats_per_member, hipStream_t st);
// flags_new[m] = flags[src[m]] (before any flag changes), then the commit
hipError_t launch_relabel_commit(const FinishArgs& f, const CommitArgs& a, hipStream_t st);

}  // namespace lbm
