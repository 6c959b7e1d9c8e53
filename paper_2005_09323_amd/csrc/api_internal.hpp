// Host-side context of the C ABI and helpers shared by the API sources.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"

namespace lbm {

constexpr int MAX_MEMBERS = 4096;
constexpr int DEFAULT_TILE = 20;  // two steps per launch while the active members fill the device, else one

struct MaskBits {
    unsigned w[MAX_MEMBERS / 32];
};

hipError_t fill_int(int* p, int n, int v, hipStream_t st);
hipError_t fill_double(double* p, int n, double v, hipStream_t st);
hipError_t set_int(int* p, int v, hipStream_t st);
// p[m] = bit m; list (if non-null) = the set members in increasing order
hipError_t set_bits(int* p, int* list, int n, const MaskBits& bits, hipStream_t st);
hipError_t fill_iota(int* p, int n, hipStream_t st);  // p[i] = i

}  // namespace lbm

struct RareScratch {
    bool ready = false;
    int blocks_per_state = 0;
    double *prefix = nullptr, *alpha = nullptr, *alpha_sum = nullptr, *scale = nullptr, *coef_w = nullptr;
    double* mass_partial = nullptr;
    int *mode = nullptr, *src = nullptr, *need_mass = nullptr, *flags_new = nullptr, *status = nullptr;
    int* status_host = nullptr;
    // relabelling clone: new block and buffer of every slot, the slots written
    long long* new_off = nullptr;
    int *new_parity = nullptr, *extra = nullptr, *n_extra = nullptr;
    // pinned read-back of the tables above (the host mirrors follow them)
    long long* new_off_host = nullptr;
    int *new_parity_host = nullptr, *n_extra_host = nullptr;
};

// What a captured chunk of lbm_step_batch depends on besides device memory:
// a replay is valid while all of it is unchanged.
struct ChunkGraphKey {
    int tile_id, one_tile, two, waves2, model, open, chunk, table_gen;
    int total_blocks, total_blocks2, compact;
    double mu, inv_sigma_dt;
    const void* ghost;
    bool operator==(const ChunkGraphKey& o) const {
        return tile_id == o.tile_id && one_tile == o.one_tile && two == o.two && waves2 == o.waves2 &&
               table_gen == o.table_gen &&
               model == o.model && open == o.open && chunk == o.chunk && total_blocks == o.total_blocks &&
               total_blocks2 == o.total_blocks2 && compact == o.compact && mu == o.mu &&
               inv_sigma_dt == o.inv_sigma_dt && ghost == o.ghost;
    }
};

struct lbm_ctx {
    int n = 0;
    std::vector<lbm_member_desc> desc;
    std::vector<lbm::MemberDev> h_members;
    lbm::MemberDev* d_members = nullptr;
    float* pop[2] = {nullptr, nullptr};
    size_t pop_floats = 0;
    float* series = nullptr;
    int cap = 0;
    double* accum = nullptr;
    hipStream_t stream = nullptr;
    // per-member bookkeeping; the host mirrors change in lockstep with the
    // device copies (same calls, same order), so no read-back is needed
    int* d_parity = nullptr;
    int* d_cursor = nullptr;
    int* d_active = nullptr;
    int* d_active_list = nullptr;  // the n_active active members in ascending order
    int n_active = 0;
    int* d_flags = nullptr;
    std::vector<int> h_parity, h_cursor, h_active;
    double* d_partial = nullptr;
    long long partial_floats = 0;
    double* d_scratch = nullptr;  // FP64 scratch for selection / mass sums
    int* d_iscratch = nullptr;    // int scratch for selection
    long long max_cells = 0;
    bool uniform_shape = true;
    int chunk = 64;
    double mu = 0.0, sigma = 1.0, dt = 1.0;
    int tile_id = lbm::DEFAULT_TILE;
    int model = 0;  // collision: 0 BGK, 1 central moments, 2 the same with unit bulk/third/fourth rates
    // open channel (every member): inlet, grid, sponge, outlet ghost columns
    bool open = false;
    float* d_ghost = nullptr;  // [member][9][ny] floats
    int max_ny = 0;
    int cu_count = 256;  // compute units of the device (the two-step kernel wants 2 workgroups per CU)
    // one-step launches: the tile shape in use (shape 0 when a two-step shape is chosen)
    int one_tile = 0;
    int nseg = 0;
    int total_blocks = 0;
    lbm::Segment seg[lbm::MAX_SEGMENTS];
    // two-step launches (when the chosen shape has two steps and every member qualifies)
    // rows per workgroup of each run of equal lattice shapes (its segment of the
    // two-step table): -1 as the shape says, 0 whole strips, else a row range
    std::vector<int> run_rows;
    int table_gen = 0;  // bumped whenever the tables are rebuilt (captured graphs hold them)
    bool two_step = false;
    bool split2 = false;  // some strip of the two-step table is split into row ranges
    int nseg2 = 0;
    int total_blocks2 = 0;
    lbm::Segment seg2[lbm::MAX_SEGMENTS];
    RareScratch rare;
    // GKTL cloning by relabelling member blocks (1, the default) or by gathering
    // every copy into the other buffer (0); both give the same states
    int relabel = 1;
    // full chunks of lbm_step_batch replay one captured HIP graph (captured on
    // a private stream, launched on `stream`)
    bool graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    ChunkGraphKey graph_key{};
    int graph_launches = 0;  // launches in the captured chunk (its parity swaps the buffers)
};

void free_rare_scratch(lbm_ctx* c);
void free_chunk_graph(lbm_ctx* c);

int lbm_fail(int code, const char* fmt, ...);
int lbm_hip_fail(hipError_t e, const char* what);
