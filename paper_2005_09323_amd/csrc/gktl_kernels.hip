// GKTL cloning (paper Appendix C.1) and the branching perturbation with mass
// rescaling (paper Appendix D), on the device.
//
// Selection runs in one workgroup: the weights are FP64, the running sum that
// the multinomial draw inverts is formed sequentially in slot order (so the
// decisions are a fixed function of the inputs), and the uniforms come from
// the counter-based Philox stream.  Cloning is a gather over the ensemble:
// every member's new state is its ancestor's, perturbed for all but the
// first copy of each ancestor.
#include "rare_kernels.hpp"

namespace lbm {

typedef float f4g __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double block_max(double v, double* sh) {
    const int t = (int)threadIdx.x, nt = (int)blockDim.x;
    sh[t] = v;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// One workgroup of 1024 threads; N <= MAX_SELECT.
__global__ __launch_bounds__(1024) void gktl_select_kernel(SelectArgs a) {
    __shared__ double sh[1024];
    __shared__ int first_slot[MAX_SELECT];
    __shared__ int n_live;
    const int t = (int)threadIdx.x, nt = (int)blockDim.x, n = a.n;
    double mx = -INFINITY;
    for (int m = t; m < n; m += nt) {
        const double s = a.k * a.accum[m];
        if (isfinite(s)) mx = fmax(mx, s);
        first_slot[m] = 0x7fffffff;
    }
    if (t == 0) n_live = 0;
    mx = block_max(mx, sh);  // max is exact and order-free
    if (!isfinite(mx)) {     // every weight non-finite: report and change nothing
        if (t == 0) *a.status = 1;
        return;
    }
    // weights relative to the largest, then the running sum in slot order
    for (int m = t; m < n; m += nt) {
        const double s = a.k * a.accum[m];
        a.prefix[m] = isfinite(s) ? exp(s - mx) : 0.0;
    }
    __syncthreads();
    if (t == 0) {
        double acc = 0.0;
        int last_live = 0;
        for (int m = 0; m < n; ++m) {
            if (isfinite(a.k * a.accum[m])) last_live = m;  // fallback ancestor if u * total rounds up to total
            acc += a.prefix[m];
            a.prefix[m] = acc;
        }
        n_live = last_live;
        *a.ln_r = mx + log(acc) - log((double)n);
        *a.status = 0;
    }
    __syncthreads();
    const double total = a.prefix[n - 1];
    for (int m = t; m < n; m += nt) {
        const U64x4 w = philox4x64_10((uint64_t)m, (uint64_t)a.period, 0, 0, a.key, PURPOSE_GKTS);
        const double target = uniform53(w.v[0]) * total;
        // first n with prefix[n] > target (prefix is non-decreasing)
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.prefix[mid] > target) hi = mid; else lo = mid + 1;
        }
        const int anc = lo < n ? lo : n_live;
        a.ancestors[m] = anc;
        atomicMin(&first_slot[anc], m);  // lowest slot taking each ancestor: order-free
    }
    __syncthreads();
    for (int m = t; m < n; m += nt) {
        const int anc = a.ancestors[m];
        const int pert = (a.n_snap > 0 && a.eps != 0.0 && first_slot[anc] != m) ? 1 : 0;
        a.mode[m] = pert ? MODE_PERTURB : MODE_COPY;
        a.src[m] = anc;
        if (pert) {
            double psum = 0.0;
            for (int q = 0; q < a.n_snap; ++q) {
                const U64x4 w = philox4x64_10((uint64_t)m, (uint64_t)a.period, (uint64_t)(q / 4), 0, a.key, PURPOSE_PRTB);
                const double al = uniform53(w.v[q % 4]);
                a.alpha[(long long)m * MAX_SNAP + q] = al;
                psum += al;
            }
            a.alpha_sum[m] = psum;
        }
    }
    __syncthreads();
    // parents of perturbed copies need their mass
    for (int m = t; m < n; m += nt) a.need_mass[m] = 0;
    __syncthreads();
    for (int m = t; m < n; m += nt)
        if (a.mode[m] == MODE_PERTURB) a.need_mass[a.src[m]] = 1;
    if (!a.relabel) return;
    // Relabelling: the first copy of each ancestor keeps the ancestor's block
    // and buffer; the k-th further copy (in slot order) takes the block of the
    // k-th state (in slot order) that left no descendant.  There are as many
    // such states as further copies, and no copy reads them.  Ranks by a
    // block-wide exclusive prefix count over slot order (each thread counts
    // PER consecutive slots, then a scan over the threads).
    constexpr int PER = MAX_SELECT / 1024;
    __shared__ int scan_dead[1024], scan_extra[1024];
    __shared__ int dead_state[MAX_SELECT];
    const int b0 = t * PER;
    int cd = 0, ce = 0;
    for (int j = 0; j < PER; ++j) {
        const int m = b0 + j;
        if (m < n) {
            cd += first_slot[m] == 0x7fffffff ? 1 : 0;
            ce += first_slot[a.ancestors[m]] != m ? 1 : 0;
        }
    }
    scan_dead[t] = cd;
    scan_extra[t] = ce;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan (Hillis-Steele)
        const int vd = t >= off ? scan_dead[t - off] : 0, ve = t >= off ? scan_extra[t - off] : 0;
        __syncthreads();
        scan_dead[t] += vd;
        scan_extra[t] += ve;
        __syncthreads();
    }
    int rd = scan_dead[t] - cd, re = scan_extra[t] - ce;  // exclusive ranks of this thread's first slot
    for (int j = 0; j < PER; ++j) {
        const int m = b0 + j;
        if (m < n && first_slot[m] == 0x7fffffff) dead_state[rd++] = m;
    }
    __syncthreads();
    for (int j = 0; j < PER; ++j) {
        const int m = b0 + j;
        if (m >= n) break;
        const int anc = a.ancestors[m];
        a.new_parity[m] = a.parity[anc];
        if (first_slot[anc] == m) {
            a.new_off[m] = a.members[anc].off;
        } else {
            a.new_off[m] = a.members[dead_state[re]].off;
            a.extra[re++] = m;
        }
    }
    if (t == 1023) *a.n_extra = scan_extra[1023];
}

// Host-chosen modes (in-place perturbation of selected members): fill the
// same tables the selection kernel fills.
__global__ void perturb_plan_kernel(PlanArgs a) {
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= a.n) return;
    const int pert = (a.mask.w[m >> 5] >> (m & 31)) & 1u;
    a.mode[m] = pert ? MODE_PERTURB : MODE_SKIP;
    a.src[m] = m;
    a.need_mass[m] = pert;
    if (pert) {
        double psum = 0.0;
        for (int q = 0; q < a.n_snap; ++q) {
            const U64x4 w = philox4x64_10((uint64_t)m, (uint64_t)a.period, (uint64_t)(q / 4), 0, a.key, PURPOSE_PRTB);
            const double al = uniform53(w.v[q % 4]);
            a.alpha[(long long)m * MAX_SNAP + q] = al;
            psum += al;
        }
        a.alpha_sum[m] = psum;
    }
}

// Sum of deviations over the fluid cells of one state, as fixed per-block
// partials (block b covers elements [b*chunk, (b+1)*chunk) of the 9*nx*ny
// floats); the partials are added in block order afterwards.
// blockIdx.y: member index (< n) or snapshot index (n + q).
__global__ __launch_bounds__(256) void mass_partial_kernel(MassArgs a) {
    const int j = (int)blockIdx.y;
    const bool snap = j >= a.n;
    if (!snap && !a.need_mass[j]) return;
    const MemberDev m = a.members[snap ? 0 : j];
    const long long plane = (long long)m.nx * m.ny;
    const long long total = 9 * plane;
    const float* base = snap ? a.snapshots + (long long)(j - a.n) * total
                             : (a.parity[j] ? a.pop1 : a.pop0) + m.off;
    __shared__ double sh[256];
    const long long b0 = (long long)blockIdx.x * MASS_CHUNK;
    double acc = 0.0;
    if (b0 < total) {
        const long long e1 = min(b0 + MASS_CHUNK, total);
        if ((m.nx & 3) == 0) {
            // four cells of one row per thread and load (a row never splits a vector)
            for (long long e = b0 + 4 * threadIdx.x; e < e1; e += 1024) {
                const f4g v = *(const f4g*)(base + e);
                const long long cell = e % plane;
                const int y = (int)(cell / m.nx), x = (int)(cell - (long long)y * m.nx);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (!in_solid(m, x + k, y)) acc += (double)v[k];
            }
        } else {
            long long e = b0 + threadIdx.x;
            // the cell of the first element by division, the next ones by stepping 256 cells on
            const long long cell = e % plane;
            int y = (int)(cell / m.nx), x = (int)(cell - (long long)y * m.nx);
            for (; e < e1; e += 256) {
                if (!in_solid(m, x, y)) acc += (double)base[e];
                x += 256;
                while (x >= m.nx) {
                    x -= m.nx;
                    if (++y == m.ny) y = 0;
                }
            }
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[(long long)j * a.blocks_per_state + blockIdx.x] = sh[0];
}

// Per perturbed member: scale s restoring the parent's mass and the
// coefficient of the rest weights, c_w = s (1 + eps sum alpha) - 1.
//   M_parent = N_fluid + sum d_parent,  M_n = N_fluid + sum d^(n),
//   M_after = M_parent + eps sum_n alpha_n M_n,  s = M_parent / M_after.
__global__ void mass_scale_kernel(ScaleArgs a) {
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= a.n || a.mode[m] != MODE_PERTURB) return;
    const double nf = a.n_fluid;
    auto mass = [&](int j) {
        double s = 0.0;
        for (int b = 0; b < a.blocks_per_state; ++b) s += a.partial[(long long)j * a.blocks_per_state + b];
        return nf + s;
    };
    const double mp = mass(a.src[m]);
    double add = 0.0;
    for (int q = 0; q < a.n_snap; ++q) add += a.alpha[(long long)m * MAX_SNAP + q] * mass(a.n + q);
    const double s = mp / (mp + a.eps * add);
    a.scale[m] = s;
    a.coef_w[m] = s * (1.0 + a.eps * a.alpha_sum[m]) - 1.0;
}

// New state of every member with mode != SKIP, written to the buffer that
// does not hold its current state:
//   copy:    d_new = d_src
//   perturb: d_new = s (d_src + eps sum_n alpha_n d^(n)) + c_w w_i
// (full populations: f_new = s (f_src + eps sum_n alpha_n f^(n)), f = w + d).
// blockIdx.y = member; each thread moves 4 consecutive floats with 16-byte
// accesses when the member block allows it (a plane of a multiple-of-4
// width never splits a vector between two directions).
// The perturbation's arithmetic, shared by every kernel that writes a
// perturbed copy (so that all of them give the same bits):
//   ad += alpha_q d^(q) (snapshots in order q = 0, 1, ...), then
//   d_new = s (d_src + eps ad) + c_w w_i, with explicit FMAs.
__device__ __forceinline__ double perturb_acc(double ad, double al, float sv) { return fma(al, (double)sv, ad); }
__device__ __forceinline__ float perturb_out(float v, double ad, double s, double eps, double cw) {
    return (float)fma(s, fma(eps, ad, (double)v), cw);
}

__global__ __launch_bounds__(256) void clone_gather_kernel(GatherArgs a) {
    const int m = (int)blockIdx.y;
    const int mode = a.mode[m];
    if (mode == MODE_SKIP) return;
    const MemberDev md = a.members[m];
    const long long plane = (long long)md.nx * md.ny;
    const long long total = 9 * plane;
    const long long e0 = 4 * ((long long)blockIdx.x * 256 + threadIdx.x);
    if (e0 >= total) return;
    const int src = a.src[m];
    const float* sp = (a.parity[src] ? a.pop1 : a.pop0) + a.members[src].off;
    float* dp = (a.parity[m] ? a.pop0 : a.pop1) + md.off;
    const bool vec = (plane & 3) == 0;
    if (vec) {
        const f4g v = *(const f4g*)(sp + e0);
        if (mode == MODE_COPY) {
            __builtin_nontemporal_store(v, (f4g*)(dp + e0));
            return;
        }
        const int i = (int)(e0 / plane);
        f4g acc = {0.0f, 0.0f, 0.0f, 0.0f};
        double ad[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < a.n_snap; ++q) {
            const double al = a.alpha[(long long)m * MAX_SNAP + q];
            const f4g sv = *(const f4g*)(a.snapshots + (long long)q * total + e0);
#pragma unroll
            for (int k = 0; k < 4; ++k) ad[k] = perturb_acc(ad[k], al, sv[k]);
        }
        const double s = a.scale[m], cw = a.coef_w[m] * WD[i], eps = a.eps;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = perturb_out(v[k], ad[k], s, eps, cw);
        *(f4g*)(dp + e0) = acc;
        return;
    }
    const int cnt = (int)min((long long)4, total - e0);
    if (mode == MODE_COPY) {
        for (int k = 0; k < cnt; ++k) dp[e0 + k] = sp[e0 + k];
        return;
    }
    const double s = a.scale[m], eps = a.eps;
    for (int k = 0; k < cnt; ++k) {
        const long long e = e0 + k;
        const int i = (int)(e / plane);
        double ad = 0.0;
        for (int q = 0; q < a.n_snap; ++q)
            ad = perturb_acc(ad, a.alpha[(long long)m * MAX_SNAP + q], a.snapshots[(long long)q * total + e]);
        dp[e] = perturb_out(sp[e], ad, s, eps, a.coef_w[m] * WD[i]);
    }
}

// Bookkeeping after a gather: members that received a new state flip parity;
// the GKTL period restarts (accum = 0) and the non-finite flag follows the state.
__global__ void clone_finish_kernel(FinishArgs a) {
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= a.n) return;
    const int mode = a.mode[m];
    if (mode == MODE_SKIP) return;
    if (a.reset_accum) {
        a.accum[m] = 0.0;
        a.flags_new[m] = a.flags[a.src[m]];
    }
}
__global__ void clone_commit_kernel(FinishArgs a) {
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= a.n || a.mode[m] == MODE_SKIP) return;
    a.parity[m] ^= 1;
    if (a.reset_accum) a.flags[m] = a.flags_new[m];
}

// Relabelling clone: the further copies extra[PLACE_GROUP * blockIdx.y + g]
// get their ancestor's state (copy) or its perturbation (the arithmetic of
// clone_gather_kernel), written into their new blocks in the ancestor's
// buffer.  A workgroup serves a group of copies over one stretch of cells, so
// that each snapshot word is read once for the whole group.  Sources are
// blocks of ancestors, destinations blocks of states without descendant:
// never the same block.
constexpr int PLACE_GROUP = 8;

__global__ __launch_bounds__(256) void clone_place_kernel(PlaceArgs a) {
    const int g0 = (int)blockIdx.y * PLACE_GROUP;
    const int ng = min(PLACE_GROUP, a.n_extra - g0);
    const MemberDev m0 = a.members[a.src[a.extra[g0]]];
    const long long plane = (long long)m0.nx * m0.ny;
    const long long total = 9 * plane;
    const long long e0 = 4 * ((long long)blockIdx.x * 256 + threadIdx.x);
    if (e0 >= total) return;
    const bool pert = a.n_snap > 0 && a.mode[a.extra[g0]] == MODE_PERTURB;  // all copies alike
    if ((plane & 3) == 0) {
        double ad[PLACE_GROUP][4];
#pragma unroll
        for (int g = 0; g < PLACE_GROUP; ++g)
#pragma unroll
            for (int k = 0; k < 4; ++k) ad[g][k] = 0.0;
        if (pert) {
            for (int q = 0; q < a.n_snap; ++q) {
                const f4g sv = *(const f4g*)(a.snapshots + (long long)q * total + e0);
#pragma unroll
                for (int g = 0; g < PLACE_GROUP; ++g) {
                    if (g >= ng) break;
                    const double al = a.alpha[(long long)a.extra[g0 + g] * MAX_SNAP + q];
#pragma unroll
                    for (int k = 0; k < 4; ++k) ad[g][k] = perturb_acc(ad[g][k], al, sv[k]);
                }
            }
        }
        const int i = (int)(e0 / plane);
        // the group's source words first: the stores below may alias them as far as
        // the compiler knows, so loads after a store would wait for it
        f4g vs[PLACE_GROUP];
#pragma unroll
        for (int g = 0; g < PLACE_GROUP; ++g) {
            if (g >= ng) break;
            const int src = a.src[a.extra[g0 + g]];
            vs[g] = *(const f4g*)((a.parity[src] ? a.pop1 : a.pop0) + a.members[src].off + e0);
        }
#pragma unroll
        for (int g = 0; g < PLACE_GROUP; ++g) {
            if (g >= ng) break;
            const int m = a.extra[g0 + g];
            float* const buf = a.parity[a.src[m]] ? a.pop1 : a.pop0;
            const f4g v = vs[g];
            f4g out = v;
            if (pert) {
                const double s = a.scale[m], cw = a.coef_w[m] * WD[i], eps = a.eps;
#pragma unroll
                for (int k = 0; k < 4; ++k) out[k] = perturb_out(v[k], ad[g][k], s, eps, cw);
            }
            __builtin_nontemporal_store(out, (f4g*)(buf + a.new_off[m] + e0));
        }
        return;
    }
    const int cnt = (int)min((long long)4, total - e0);
    for (int g = 0; g < ng; ++g) {
        const int m = a.extra[g0 + g];
        const int src = a.src[m];
        float* const buf = a.parity[src] ? a.pop1 : a.pop0;
        const float* sp = buf + a.members[src].off;
        float* dp = buf + a.new_off[m];
        for (int k = 0; k < cnt; ++k) {
            const long long e = e0 + k;
            if (!pert) {
                dp[e] = sp[e];
                continue;
            }
            const int i = (int)(e / plane);
            double ad = 0.0;
            for (int q = 0; q < a.n_snap; ++q)
                ad = perturb_acc(ad, a.alpha[(long long)m * MAX_SNAP + q], a.snapshots[(long long)q * total + e]);
            dp[e] = perturb_out(sp[e], ad, a.scale[m], a.eps, a.coef_w[m] * WD[i]);
        }
    }
}

// After the relabelling clone: every slot's block, buffer and flag.
__global__ void clone_relabel_commit_kernel(CommitArgs a) {
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= a.n) return;
    a.members[m].off = a.new_off[m];
    a.parity[m] = a.new_parity[m];
    a.accum[m] = 0.0;
    a.flags[m] = a.flags_new[m];
}

hipError_t launch_place(const PlaceArgs& a, long long floats_per_member, hipStream_t st) {
    if (a.n_extra == 0) return hipSuccess;
    const unsigned gx = (unsigned)((floats_per_member / 4 + 255) / 256 + 1);
    hipLaunchKernelGGL(clone_place_kernel, dim3(gx, (a.n_extra + PLACE_GROUP - 1) / PLACE_GROUP), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_relabel_commit(const FinishArgs& f, const CommitArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(clone_finish_kernel, dim3((f.n + 255) / 256), dim3(256), 0, st, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(clone_relabel_commit_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_select(const SelectArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(gktl_select_kernel, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_plan(const PlanArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(perturb_plan_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_mass(const MassArgs& a, int n_states, hipStream_t st) {
    hipLaunchKernelGGL(mass_partial_kernel, dim3(a.blocks_per_state, n_states), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_scale(const ScaleArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(mass_scale_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_gather(const GatherArgs& a, long long floats_per_member, hipStream_t st) {
    const unsigned gx = (unsigned)((floats_per_member / 4 + 255) / 256 + 1);
    hipLaunchKernelGGL(clone_gather_kernel, dim3(gx, a.n), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_finish(const FinishArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(clone_finish_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(clone_commit_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lbm
