// Internal launchers shared by the C-ABI wrappers and the multi-step driver.
#pragma once

#include <hip/hip_ext.h>

#include "common.hpp"

namespace trk {

// Start/stop events carried by the next timed dispatch of this host thread
// (set for one launcher call by a TimedDispatch scope).  The dispatch packet
// records them itself (hipExtLaunchKernelGGL), so their elapsed time is the
// kernel's execution alone, without the queueing around it.
struct DispatchEvents {
    hipEvent_t t0 = nullptr, t1 = nullptr;
};
inline thread_local DispatchEvents g_dispatch_events;
struct TimedDispatch {
    TimedDispatch(hipEvent_t t0, hipEvent_t t1) { g_dispatch_events = DispatchEvents{t0, t1}; }
    ~TimedDispatch() { g_dispatch_events = DispatchEvents{}; }
    TimedDispatch(const TimedDispatch&) = delete;
    TimedDispatch& operator=(const TimedDispatch&) = delete;
};
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, size_t shm, hipStream_t st, Args... args) {
    DispatchEvents& ev = g_dispatch_events;
    if (ev.t0 || ev.t1) {
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shm, st, ev.t0, ev.t1, 0u, args...);
        ev = DispatchEvents{};
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
    }
}

// Fiber source: the tensor in the strides of the descriptor, and optional
// mode-major replicas (X_[n] column-major) that make every fiber contiguous.
struct XSrc {
    const void* X;
    const void* rep[kMaxOrder];
};

struct Shape {
    int maxI = 0, maxR = 0, maxRR = 0;
    int64_t maxJ = 0;
};
Shape shape_of(const tr_desc& d);

tr_status validate_desc(const tr_desc* d);
int dtype_size(int dt);

// a3/a4: draw (optionally) and build sampled subchain rows (optionally).
hipError_t launch_sample_subchain(const tr_desc& d, ModeSrc ms, int m, CdfPtrs cdf,
                                  const uint64_t* cdf_J, int stream_tag, Ptrs cores,
                                  int32_t* idx, double* pF, void* S, bool do_sample,
                                  bool do_subchain, hipStream_t st);
// sample_mode 0: indices given in idx; 1: drawn; 2: every column of X_[n]
// once (m = J_n, p = 1/J_n, column order of the cyclic unfolding).
hipError_t launch_sample_subchain_mode(const tr_desc& d, ModeSrc ms, int m, CdfPtrs cdf,
                                       const uint64_t* cdf_J, int stream_tag, Ptrs cores,
                                       int32_t* idx, double* pF, void* S, int sample_mode,
                                       bool do_subchain, hipStream_t st);

// Row tile and sample group of a gradient block, XCD-aware.  Workgroups go
// to the eight XCDs round-robin by linear id (block b on XCD b mod 8), each
// with its own L2; the T row tiles of a sample group take consecutive slots
// of one XCD, so the group's rows of S are fetched into that L2 once and
// read from there by the other tiles.  With fewer than eight groups (XCDs
// would idle) the blocks keep the plain order.  Grid: xcd_grid(T, G)
// blocks; false for the padding blocks past the last group (they exit at
// once).
inline unsigned xcd_grid(int T, int G) {
    return G >= 8 ? 8u * (unsigned)T * (unsigned)((G + 7) / 8) : (unsigned)(T * G);
}
__device__ inline bool xcd_tile_group(int T, int G, int& tile, int& grp) {
    const int b = (int)blockIdx.x;
    if (G < 8) {
        grp = b / T;
        tile = b - grp * T;
        return true;
    }
    const int slot = b >> 3, gl = slot / T;
    tile = slot - gl * T;
    grp = (b & 7) + 8 * gl;
    return grp < G;
}

// a5/a6: partial gradients and loss.  Layout of the workspace returned by
// grad_ws_layout.
struct GradWs {
    size_t gpart_off, lpart_off, total;
    int groups, row_tiles, ti, tf;
};
GradWs grad_ws_layout(const tr_desc& d, int m, int prec);
// tf: samples per staged chunk (64, or 128 for at most 8 column tiles).
hipError_t launch_grad_mfma_f32(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx,
                                const float* S, const double* pF, int m, int groups, int row_tiles, float* gp,
                                double* lp, int tf, hipStream_t st);
hipError_t launch_grad_mixed(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                             const double* pF, int m, int prec, int groups, int row_tiles, float* gp, double* lp,
                             hipStream_t st);
hipError_t launch_grad_partial(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs,
                               const int32_t* idx, const void* S, const double* pF, int m,
                               int prec, void* ws, const GradWs& L, hipStream_t st);

// Per-block loss partials of the gradient kernels: part[g * tiles_max + b]
// for sample group g and row tile b < ceil(I_n / ti).
struct LossParts {
    const double* part;
    int groups, tiles_max, ti;
};
// Their sum in a fixed order (strided per thread, then the block tree);
// valid in every thread.  ``red`` needs blockDim/64 entries.
__device__ inline double loss_parts_sum(const LossParts& lp, int In, double* red) {
    const int rt = (In + lp.ti - 1) / lp.ti;
    const int tot = lp.groups * rt;
    double s = 0.0;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int g = i / rt, b = i - g * rt;
        s += lp.part[(int64_t)g * lp.tiles_max + b];
    }
    return block_sum(s, red);
}

// Step-counter advance folded into the last kernel of a step.  When the
// kernel's blocks use t (t_read: the Robbins-Monro rule), every block counts
// itself in ``ctr`` once it is done and the last one resets ``ctr`` and adds
// 1 to ``t``.  No fence is needed: a block's read of t has completed before
// its count (its addresses depend on the mode drawn from t), the counter and
// t change only through device-scope atomics, and the kernels that read t
// next start after this kernel has ended.  (An agent-scope fence here would
// write back the L2 once per block.)  Otherwise every other reader of t in
// the step has finished before the kernel starts (its blocks take the mode
// from the published slot and ignore t), and one block adds 1 at once.
// Disabled when t is null.
struct StepBump {
    uint64_t* t;
    unsigned* ctr;
};
__device__ inline void bump_if_last(const StepBump& b, bool t_read) {
    if (!b.t) return;
    if (!t_read) {   // no block uses t: one block advances it, nobody waits
        if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(b.t), 1ull);
        return;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
        if (atomicAdd(b.ctr, 1u) == nb - 1) {
            atomicExch(b.ctr, 0u);
            atomicAdd(reinterpret_cast<unsigned long long*>(b.t), 1ull);
        }
    }
}

// Reduce partials into g (core dtype) and the loss; optionally apply the
// plain direction p = -g with ``rule`` to the core in place.
hipError_t launch_grad_reduce(const tr_desc& d, ModeSrc ms, const void* ws, const GradWs& L,
                              void* g, double* loss, bool apply, MutPtrs cores, MutPtrs accum,
                              tr_step rule, int32_t* status, hipStream_t st, StepBump step = StepBump{});

// FP64-accumulated Gram S^T diag(1/(m J_n pF)) S.
struct GramWs {
    size_t part_off, total;
    int groups, tiles;
};
GramWs gram_ws_layout(const tr_desc& d, int m);
// ``mid`` (optional) is recorded between the per-group sums and their
// reduction.
// With S null and pF null: the unweighted Gram G_{n(2)}^T G_{n(2)} of the
// step's core, rows taken from ``rows`` (m ignored; L laid out for maxI).
hipError_t launch_gram(const tr_desc& d, ModeSrc ms, const void* S, const double* pF, int m,
                       double* gram, void* ws, const GramWs& L, hipStream_t st, hipEvent_t mid = nullptr,
                       Ptrs rows = Ptrs{});

// a7/a8: Cholesky of gram + damping (with fallback) then solve and update.
struct UpdWs {
    size_t L_off, dinv_off, flag_off, total;
};
UpdWs upd_ws_layout(const tr_desc& d);
hipError_t launch_scaled_update(const tr_desc& d, ModeSrc ms, const double* gram, Damp damping,
                                const void* g, MutPtrs cores, MutPtrs accum, tr_step rule,
                                int32_t* status, void* ws, const UpdWs& L, hipStream_t st);
// The same for RR <= 128 through the blocked sweep (g already reduced).
bool sweep_supported(const tr_desc& d);
hipError_t launch_sweep_update(const tr_desc& d, ModeSrc ms, const double* gram, Damp damping, const void* g,
                               double* loss, MutPtrs cores, MutPtrs accum, tr_step rule, int32_t* status, void* ws,
                               const UpdWs& L, StepBump step, hipStream_t st);
// The two halves: -(gram + damping I)^{-1} (one workgroup) and the
// row-parallel p = g (-M^{-1}) with the rule.
hipError_t launch_sweep_inverse(const tr_desc& d, ModeSrc ms, const double* gram, Damp damping, const UpdWs& L,
                                void* ws, int32_t* status, hipStream_t st, double rank_tol = 0.0);
hipError_t launch_sweep_apply(const tr_desc& d, ModeSrc ms, const void* g, LossParts lp, double* loss, MutPtrs cores,
                              MutPtrs accum, tr_step rule, int32_t* status, void* ws, const UpdWs& L, StepBump step,
                              hipStream_t st);
hipError_t launch_plain_update(const tr_desc& d, ModeSrc ms, const void* g, MutPtrs cores,
                               MutPtrs accum, tr_step rule, int32_t* status, hipStream_t st);

// a2: laws.
size_t dist_ws_bytes(const tr_desc& d, int law);
// bump (optional): the step counter the law's last kernel advances.
hipError_t launch_dist(const tr_desc& d, ModeSrc ms, bool use_mode, int k, int law, Ptrs cores,
                       uint64_t* const* cdf_out, int32_t* status, void* ws, hipStream_t st,
                       uint64_t* bump = nullptr);
size_t dist_opt_ws_bytes(const tr_desc& d);
hipError_t launch_dist_optimal(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs,
                               uint64_t* cdf_J, int32_t* status, void* ws, hipStream_t st);

hipError_t launch_bump(uint64_t* t_dev, hipStream_t st);

// a11: batched independent problems.
size_t batch_lds_bytes(int chunk);
hipError_t launch_batch_steps(const tr_batch_item* items, int count, int steps, int chunk, int waves, hipStream_t st);
size_t batch_split_ws_bytes(int count, int splits);
hipError_t launch_batch_split(const tr_batch_item* items, int count, int steps, int chunk, int waves, int splits,
                              void* ws, hipStream_t st);
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st);

}  // namespace trk

namespace trk {
size_t relerr_ws_bytes(const tr_desc& d);
hipError_t launch_relerr(const tr_desc& d, Ptrs cores, const void* Xt, double xnorm2, double* rse, void* ws,
                         hipStream_t st);
hipError_t launch_reconstruct(const tr_desc& d, Ptrs cores, void* Xo, hipStream_t st);
hipError_t launch_replicate(const tr_desc& d, const void* X, int n, void* Xn, hipStream_t st);
}  // namespace trk
