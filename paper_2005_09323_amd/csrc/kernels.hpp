// Kernel argument blocks and launchers shared between the kernel sources and
// the C-ABI layer.
#pragma once

#include "common.hpp"

namespace lbm {

constexpr int MAX_SEGMENTS = 32;  // runs of consecutive members with one lattice shape
constexpr int MAX_CHUNK = 256;    // steps per drag-reduction chunk

struct Segment {
    int block_begin;       // first workgroup of the segment
    int member_begin;      // first member
    int tiles_per_member;  // tiles_x * tiles_y
    int tiles_x;           // tiles of 256 columns
    int vec;               // 1: width a multiple of 4, rows handled four cells per lane
    int rows;              // two-step strips: rows per workgroup (the lattice height when not split)
};

struct StepArgs {
    const MemberDev* members;
    const int* parity;   // per member: which buffer holds its state before this chunk
    const int* active;
    float* pop0;
    float* pop1;
    double* partial;     // drag partials [member][slot][ring]
    int slot;            // step index within the chunk
    int flip;            // slot & 1: parity of this step relative to the chunk start
    int xcd;             // remap workgroups so each XCD gets contiguous tiles
    int total_blocks;
    int nseg;
    Segment seg[MAX_SEGMENTS];
    // non-null: the launch covers only these members (all of seg[0]'s shape),
    // tiles_per_member workgroups each, in list order
    const int* active_list;
    // two-step launches: 1 when some strip is split into row ranges (Segment::rows)
    int split;
    // non-null: open channels; the outlet ghost columns [member][9][ny]
    // (MemberDev::ghost_off), filled for this step by the ghost kernel
    const float* ghost;
};

struct GhostArgs {
    const MemberDev* members;
    const int* parity;
    const int* active;
    const float* pop0;
    const float* pop1;
    float* ghost;
    int flip;            // parity of the step's source buffer relative to the chunk start
};

struct InitArgs {
    const MemberDev* members;
    float* pop0;
    double* partial;
    uint64_t seed;
    double noise_amp;
    double ux0;  // initial uniform x-velocity
};

struct FinalizeArgs {
    const MemberDev* members;
    const int* active;
    int* parity;
    int* cursor;
    int* flags;
    const double* partial;
    float* series;
    double* accum;
    long long ld;        // row stride of the drag series
    int n;               // steps in this chunk
    int accumulate;      // add the observable to accum (0 for step 0)
    int swap_parity;     // parity of the number of buffer swaps in this chunk (one per kernel launch)
    double mu;
    double inv_sigma_dt; // dt / sigma
};

struct TileShape {
    int tyt;    // waves per workgroup
    int r;      // rows per wave (a tile is 256 columns by tyt * r rows); 1 for two-step shapes
    int xcd;    // 1: remap workgroups so each XCD gets a contiguous range of tiles
    int steps;  // lattice steps per launch: 1, or 2 (a strip of 256 columns swept bottom to top)
    int adaptive;  // two-step shape used only while the active members give a strip per CU
    int seg_rows;  // two-step shapes: rows per workgroup (0: whole strips; -1: split only when
                   // the strips alone leave workgroup slots empty)
};

extern const TileShape TILE_SHAPES[];
extern const int N_TILE_SHAPES;

// model: 0 BGK, 1 central moments (every member of the launch uses it)
hipError_t launch_step(int tile_id, const StepArgs& a, int model, hipStream_t st);
// two steps per launch, `waves` rows per iteration; the segment table must
// describe strips of 256 columns (tiles_per_member = tiles_x = nx / 256)
hipError_t launch_step2(int waves, const StepArgs& a, int model, hipStream_t st);
hipError_t launch_init(const InitArgs& a, int n_members, long long max_cells, hipStream_t st);
// the outlet ghost columns of the open-channel members for the next one-step launch
hipError_t launch_outlet_ghost(const GhostArgs& a, int n_members, int max_ny, hipStream_t st);
hipError_t launch_finalize(const FinalizeArgs& a, int n_members, hipStream_t st);

}  // namespace lbm
