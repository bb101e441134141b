// a10: sampled-entry loss L = 1/(2B) sum_b (Trace(G_0(i_0^b) ... G_{N-1}(i_{N-1}^b)) - x_b)^2
// and its gradient with respect to every core.
//
// Forward: one thread per (entry b, row s of the ring product), the row
// carried through the N slices in registers; the diagonal entries are
// summed per entry in LDS.  Only the residuals leave the kernel.
//
// Backward: dTrace/dG_k(i_k) = M_{!=k}^T with M_{!=k} = G_{k+1}(i_{k+1}) ...
// G_{k-1}(i_{k-1}), i.e. the row of G^{!=k}_[2] at entry b (the block
// gradient of eq:gradient restricted to sampled entries).  Every M_{!=k} is
// recomputed from the slices (nothing from the forward is kept but the
// residuals): one thread per (entry, core k, row of M_{!=k}).  Contributions
// of a block's entries are added in entry order into a block-private slice of
// the workspace, each gradient position owned by one thread; two more
// kernels add the block slices in a fixed order.  No float atomics: results
// are bitwise reproducible.
#include <algorithm>

#include "internal.hpp"

namespace trk {

constexpr int kEntBlock = 256;

// Row ``s`` of A_{k0} A_{k0+1} ... (``len`` slices cyclically from k0) for
// entry idx.  RM bounds every rank (loops have fixed trip counts); slice
// entries are loaded at clamped in-bounds indices and the products masked
// afterwards, so no load waits behind a branch and a slice's loads are all
// in flight together.  v[c] = 0 for c >= the row's length.
template <int RM>
__device__ inline void chain_row(const tr_desc& d, const Ptrs& cores, const int32_t* ik, int k0, int len, int s,
                                 float* v) {
    const int N = d.N;
    int k = k0;
    {
        const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
        const float* A = static_cast<const float*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
#pragma unroll
        for (int c = 0; c < RM; ++c) {
            const float a = A[s + Rk * (c < Rk1 ? c : Rk1 - 1)];
            v[c] = c < Rk1 ? a : 0.f;
        }
    }
    for (int q = 1; q < len; ++q) {
        k = ring_next(k, N);
        const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
        const float* A = static_cast<const float*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
        float w[RM];
#pragma unroll
        for (int c = 0; c < RM; ++c) {
            const float* col = A + Rk * (c < Rk1 ? c : Rk1 - 1);
            float a[RM];
#pragma unroll
            for (int r = 0; r < RM; ++r) a[r] = col[r < Rk ? r : Rk - 1];
            float acc = 0.f;
#pragma unroll
            for (int r = 0; r < RM; ++r) acc += r < Rk ? v[r] * a[r] : 0.f;
            w[c] = c < Rk1 ? acc : 0.f;
        }
#pragma unroll
        for (int c = 0; c < RM; ++c) v[c] = w[c];
    }
}

// Rank bound of the entry kernels: the largest R_k rounded up to 4, 8, 12 or 16.
static inline int rank_bound(const tr_desc& d) {
    int mr = 0;
    for (int k = 0; k < d.N; ++k) mr = d.R[k] > mr ? d.R[k] : mr;
    return mr <= 4 ? 4 : (mr <= 8 ? 8 : (mr <= 12 ? 12 : 16));
}

template <typename TX, int RM>
__global__ __launch_bounds__(kEntBlock) void k_entry_fwd(tr_desc d, Ptrs cores, const int32_t* __restrict__ idx,
                                                         const TX* __restrict__ x, int B, float* __restrict__ resid,
                                                         double* __restrict__ part) {
    const int N = d.N, R0 = d.R[0];
    const int per = kEntBlock / R0;
    const int lb = threadIdx.x / R0, s = threadIdx.x % R0;
    const int64_t b = (int64_t)blockIdx.x * per + lb;
    __shared__ float diag[kEntBlock];
    float mine = 0.f;
    if (lb < per && b < B) {
        int ik[kMaxOrder];
        bool ok = true;
        for (int k = 0; k < N; ++k) {
            ik[k] = idx[b * N + k];
            if (ik[k] < 0 || ik[k] >= d.I[k]) ok = false;
        }
        if (ok) {
            float v[RM];
            chain_row<RM>(d, cores, ik, 0, N, s, v);
#pragma unroll
            for (int c = 0; c < RM; ++c)
                if (c == s) mine = v[c];
        } else {
            mine = NAN;   // invalid caller index
        }
    }
    diag[threadIdx.x] = mine;
    __syncthreads();
    double sq = 0.0;
    if (s == 0 && lb < per && b < B) {
        float tr_ = 0.f;
        for (int q = 0; q < R0; ++q) tr_ += diag[threadIdx.x + q];
        const float r = tr_ - (float)to_f64(x[b]);
        resid[b] = r;
        sq = (double)r * (double)r;
    }
    __shared__ double red[kEntBlock / 64];
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// loss = 1/(2B) sum of the forward's block partials: strided per thread in
// block order, then the block tree (a fixed order).
__global__ __launch_bounds__(256) void k_entry_loss(const double* __restrict__ part, int nb, int B, double* loss) {
    __shared__ double red[4];
    double s = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) s += part[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *loss = s / (2.0 * (double)B);
}

// LDS layout of the backward: every slice zero-padded to RM x RM (entry
// (r, c) at r + RM c) and followed by one float of padding, the entry stride
// odd, so that the slices of one entry and the entries of a chunk start in
// different LDS banks.
template <int RM>
struct EntLds {
    static constexpr int SS = RM * RM + 1;
    __host__ __device__ static int es(int N) { return (N * SS) | 1; }
};

// Backward, phase 1: per block of EPB entries, in slabs of PF entries whose
// indices and scaled residuals are read once, and chunks of SB entries:
// (i) the chunk's slices are staged in LDS (padded as above; an entry with an
// invalid index is staged from row 0 and skipped); (ii) one thread per
// (entry, core k, row s of M_{!=k}) carries the row through the N-1 other
// slices at fixed offsets (the zero padding keeps the products exact for any
// ranks <= RM) and writes resid * row into the chunk's contributions, laid
// out like the slices; (iii) one thread per gradient position (k, a, b) adds
// the chunk's contributions to the block's private gradient slice in entry
// order.  SLICE_LDS: the slice is accumulated in LDS and written out once;
// the order of the additions, hence the result, is the same either way.
template <bool SLICE_LDS, int RM>
__global__ __launch_bounds__(1024) void k_entry_bwd_acc(tr_desc d, Ptrs cores, const int32_t* __restrict__ idx,
                                                        const float* __restrict__ resid, int B, int EPB, int SB,
                                                        int PF, float scale, const double* __restrict__ dscale,
                                                        float* __restrict__ gpart, int64_t slice_len) {
    constexpr int SS = EntLds<RM>::SS, RM2 = RM * RM;
    const int N = d.N, ES = EntLds<RM>::es(N), BT = blockDim.x, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* sl = reinterpret_cast<float*>(smem_raw);              // [SB][ES] staged slices
    float* cb = sl + (size_t)SB * ES;                             // [SB][ES] contributions
    int* sidx = reinterpret_cast<int*>(cb + (size_t)SB * ES);     // [PF][N]; first index -1: entry skipped
    float* sres = reinterpret_cast<float*>(sidx + PF * N);        // [PF] scaled residuals
    float* Gout = gpart + (int64_t)blockIdx.x * slice_len;
    float* G = SLICE_LDS ? sres + PF : Gout;                      // [slice_len]
    for (int64_t e = tid; e < slice_len; e += BT) G[e] = 0.f;
    // dL/dG_k of L = 1/(2B) sum r^2: the 1/B of the mean applied here
    const float sc = (float)((double)scale * (dscale ? *dscale : 1.0) / (double)B);
    const int64_t b0 = (int64_t)blockIdx.x * EPB;
    const int64_t b1 = min((int64_t)B, b0 + EPB);
    for (int64_t ps = b0; ps < b1; ps += PF) {
        const int np = (int)min((int64_t)PF, b1 - ps);
        __syncthreads();   // the previous slab is done with sidx and sres
        for (int lb = tid; lb < np; lb += BT) {
            bool ok = true;
            for (int k = 0; k < N; ++k) {
                const int v = idx[(ps + lb) * N + k];
                ok = ok && v >= 0 && v < d.I[k];
                sidx[lb * N + k] = v;
            }
            if (!ok) sidx[lb * N] = -1;
            sres[lb] = resid[ps + lb] * sc;
        }
        for (int cs = 0; cs < np; cs += SB) {
            const int nb = min(SB, np - cs);
            const int* cidx = sidx + cs * N;
            __syncthreads();   // indices ready; the previous chunk is done with sl and cb
            // (i) staging: eight loads per thread issued together per pass, at
            // clamped positions, then stored
            constexpr int kStagePer = 8;
            const int tot = nb * N * RM2;
            for (int e0 = 0; e0 < tot; e0 += kStagePer * BT) {
                float v[kStagePer];
                int so[kStagePer];
#pragma unroll
                for (int u = 0; u < kStagePer; ++u) {
                    const int e = e0 + u * BT + tid;
                    const int ec = e < tot ? e : tot - 1;
                    const int lb = ec / (N * RM2), rem = ec - lb * (N * RM2);
                    const int kk = rem / RM2, q = rem - kk * RM2, r = q % RM, c = q / RM;
                    const int Rk = d.R[kk], Rk1 = d.R[ring_next(kk, N)];
                    const bool in = cidx[lb * N] >= 0 && r < Rk && c < Rk1;
                    const gptr<float> src = lane_pick_global<float>(cores.p, kk);   // kk may differ across lanes
                    const float a = src[in ? (int64_t)cidx[lb * N + kk] * Rk * Rk1 + r + Rk * c : 0];
                    v[u] = in ? a : 0.f;
                    so[u] = lb * ES + kk * SS + q;
                }
#pragma unroll
                for (int u = 0; u < kStagePer; ++u)
                    if (e0 + u * BT + tid < tot) sl[so[u]] = v[u];
            }
            __syncthreads();
            // (ii) contributions
            const int tc = nb * N * RM;
            for (int e = tid; e < tc; e += BT) {
                const int lb = e / (N * RM), rem = e - lb * (N * RM), k = rem / RM, s = rem - k * RM;
                const int k0 = ring_next(k, N);
                if (s >= d.R[k0] || cidx[lb * N] < 0) continue;
                const float* base = sl + lb * ES;
                float v[RM];
                {
                    const float* A = base + k0 * SS + s;
#pragma unroll
                    for (int c = 0; c < RM; ++c) v[c] = A[RM * c];
                }
                int kk = k0;
                for (int q = 2; q < N; ++q) {
                    kk = ring_next(kk, N);
                    const float* A = base + kk * SS;
                    float w[RM];
#pragma unroll
                    for (int c = 0; c < RM; ++c) {
                        float acc = 0.f;
#pragma unroll
                        for (int r = 0; r < RM; ++r) acc += v[r] * A[r + RM * c];
                        w[c] = acc;
                    }
#pragma unroll
                    for (int c = 0; c < RM; ++c) v[c] = w[c];
                }
                const float rv = sres[cs + lb];
                float* out = cb + lb * ES + k * SS + RM * s;
#pragma unroll
                for (int c = 0; c < RM; ++c) out[c] = rv * v[c];
            }
            __syncthreads();
            // (iii) ordered accumulation: each thread owns gradient positions
            // (k, c, s) and adds the chunk's entries to them in entry order
            for (int p = tid; p < N * RM2; p += BT) {
                const int k = p / RM2, q = p - k * RM2, c = q % RM, s = q / RM;
                const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
                if (c >= Rk || s >= Rk1) continue;
                int64_t go = 0;
                for (int j = 0; j < k; ++j) go += (int64_t)d.I[j] * d.R[j] * d.R[ring_next(j, N)];
                float* Gk = G + go + c + Rk * s;
                const float* src = cb + k * SS + q;
                const int RRk = Rk * Rk1;
                for (int lb = 0; lb < nb; ++lb)
                    if (cidx[lb * N] >= 0) Gk[(int64_t)cidx[lb * N + k] * RRk] += src[lb * ES];
            }
        }
    }
    if (SLICE_LDS) {
        __syncthreads();
        for (int64_t e = tid; e < slice_len; e += BT) Gout[e] = G[e];
    }
}

// Backward, phase 2: the block slices summed in a fixed order, in two levels
// for parallelism.  Level 1: thread per element, grid row g sums run g of QG
// consecutive runs of block slices.  Level 2: the run totals in run order,
// into grads[k].
__global__ __launch_bounds__(256) void k_entry_bwd_reduce1(const float* __restrict__ gpart, int nblocks, int QG,
                                                           int64_t slice_len, float* __restrict__ red) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= slice_len) return;
    const int g = blockIdx.y;
    const int q0 = (int)((int64_t)nblocks * g / QG), q1 = (int)((int64_t)nblocks * (g + 1) / QG);
    float s = 0.f;
#pragma unroll 8
    for (int q = q0; q < q1; ++q) s += gpart[(int64_t)q * slice_len + e];
    red[(int64_t)g * slice_len + e] = s;
}

__global__ __launch_bounds__(256) void k_entry_bwd_reduce2(tr_desc d, const float* __restrict__ red, int QG,
                                                           int64_t slice_len, MutPtrs grads) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= slice_len) return;
    int k = 0;
    int64_t base = 0;
    for (; k < d.N; ++k) {
        const int64_t len = (int64_t)d.I[k] * d.R[k] * d.R[ring_next(k, d.N)];
        if (e < base + len) break;
        base += len;
    }
    float s = 0.f;
#pragma unroll 8
    for (int g = 0; g < QG; ++g) s += red[(int64_t)g * slice_len + e];
    static_cast<float*>(grads.p[k])[e - base] = s;
}

struct EntryPlan {
    int fwd_blocks, bwd_blocks, bwd_threads, EPB, SB, PF, QG;
    int64_t slice_len;
    size_t part_off, gpart_off, red_off, total, bwd_shm;
    bool slice_lds;   // the block's gradient slice fits in LDS beside the staging
};

// Blocks of the backward: two per compute unit of a 256-CU device when there
// are enough entries, fewer when the private slices would pass 64 MB.
static EntryPlan entry_plan(const tr_desc& d, int B) {
    EntryPlan P{};
    const int per = kEntBlock / d.R[0];
    P.fwd_blocks = (B + per - 1) / per;
    int64_t sl = 0;
    for (int k = 0; k < d.N; ++k) sl += (int64_t)d.I[k] * d.R[k] * d.R[ring_next(k, d.N)];
    P.slice_len = sl;
    const int RM = rank_bound(d), SS = RM * RM + 1, ES = (d.N * SS) | 1;
    const int cap_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(512, ((int64_t)64 << 20) / (sl * 4)));
    int blocks = std::min(cap_blocks, (B + 7) / 8);
    P.EPB = (B + blocks - 1) / blocks;
    P.bwd_blocks = (B + P.EPB - 1) / P.EPB;
    P.PF = std::min(P.EPB, 64);
    const size_t pf_bytes = (size_t)P.PF * (d.N + 1) * 4;
    const size_t per_entry = (size_t)2 * ES * 4;   // staged slices + contributions
    P.slice_lds = (size_t)sl * 4 <= 40 * 1024 && (size_t)sl * 4 + pf_bytes + per_entry + 64 <= 64 * 1024;
    const size_t avail = 64 * 1024 - 64 - pf_bytes - (P.slice_lds ? (size_t)sl * 4 : 0);
    int SB = 32;
    while (SB > 1 && (size_t)SB * per_entry > avail) SB >>= 1;
    P.SB = SB;
    P.bwd_shm = (size_t)SB * per_entry + pf_bytes + (P.slice_lds ? (size_t)sl * 4 : 0);
    const int pos = d.N * RM * RM;
    P.bwd_threads = std::min(1024, std::max(256, (pos + 63) / 64 * 64));
    P.QG = std::max(1, std::min(32, (P.bwd_blocks + 15) / 16));
    P.part_off = 0;
    P.gpart_off = align_up((size_t)P.fwd_blocks * 8);
    P.red_off = P.gpart_off + align_up((size_t)P.bwd_blocks * sl * 4);
    P.total = P.red_off + align_up((size_t)P.QG * sl * 4);
    return P;
}

// ------------------------------------------------------------ completion --
//
// Tensor completion with a ridge term on the sampled-entry loss: per step,
// B observed entries drawn uniformly with replacement (position
// floor(r |Omega| / 2^64), r from Philox counter (t, b, 0, TR_STREAM_ENTRY)),
// the forward and backward above, then G_k <- rule(G_k, p) with
// p = -(dL/dG_k + lambda G_k) for every core, or for core n = the step's
// mode only.

template <typename TX>
__global__ __launch_bounds__(256) void k_completion_draw(tr_desc d, const uint64_t* __restrict__ t_dev,
                                                         uint64_t seed, const int32_t* __restrict__ obs_idx,
                                                         const TX* __restrict__ obs_x, int64_t n_obs, int B,
                                                         int32_t* __restrict__ bidx, TX* __restrict__ bx) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const uint64_t t = *t_dev;
    const int64_t j = (int64_t)mulhi64(draw_word(seed, t, (uint64_t)b, 0, TR_STREAM_ENTRY), (uint64_t)n_obs);
    for (int k = 0; k < d.N; ++k) bidx[(int64_t)b * d.N + k] = obs_idx[j * d.N + k];
    bx[b] = obs_x[j];
}

// loss = 1/(2B) sum r^2 (the forward's block partials, in block order) +
// lambda/2 sum_k ||G_k||^2 (each strided per thread, then the block tree).
__global__ __launch_bounds__(256) void k_completion_loss(tr_desc d, const double* __restrict__ part, int nb, int B,
                                                         Ptrs cores, double lam, double* __restrict__ loss) {
    __shared__ double red[4];
    double s = 0.0;
    if (lam != 0.0)
        for (int k = 0; k < d.N; ++k) {
            const float* G = static_cast<const float*>(cores.p[k]);
            const int64_t len = (int64_t)d.I[k] * d.R[k] * d.R[ring_next(k, d.N)];
            for (int64_t e = threadIdx.x; e < len; e += blockDim.x) s += (double)G[e] * (double)G[e];
        }
    const double ridge = block_sum(s, red);
    double data = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) data += part[q];
    data = block_sum(data, red);
    if (threadIdx.x == 0) *loss = data / (2.0 * (double)B) + 0.5 * lam * ridge;
}

__global__ __launch_bounds__(256) void k_completion_update(tr_desc d, const uint64_t* __restrict__ t_dev,
                                                           uint64_t seed, int block, MutPtrs cores, MutPtrs accum,
                                                           const float* __restrict__ grads, int64_t slice_len,
                                                           double lam, tr_step rule, int32_t* status) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= slice_len) return;
    const uint64_t t = *t_dev;
    int k = 0;
    int64_t base = 0;
    for (; k < d.N; ++k) {
        const int64_t len = (int64_t)d.I[k] * d.R[k] * d.R[ring_next(k, d.N)];
        if (e < base + len) break;
        base += len;
    }
    if (block && k != pick_mode(seed, t, d.N)) return;
    float* G = static_cast<float*>(cores.p[k]);
    float* A = static_cast<float*>(accum.p[k]);
    const int64_t o = e - base;
    const double p = -((double)grads[e] + lam * (double)G[o]);
    apply_rule(G, A, o, p, rule, t, status);
}

template <typename TX>
static void launch_entry_fwd(const tr_desc& d, Ptrs cp, const int32_t* idx, const TX* x, int B, float* resid,
                             double* part, int blocks, hipStream_t st) {
    switch (rank_bound(d)) {
        case 4: hipLaunchKernelGGL((k_entry_fwd<TX, 4>), dim3(blocks), dim3(kEntBlock), 0, st, d, cp, idx, x, B, resid,
                                   part); break;
        case 8: hipLaunchKernelGGL((k_entry_fwd<TX, 8>), dim3(blocks), dim3(kEntBlock), 0, st, d, cp, idx, x, B, resid,
                                   part); break;
        case 12: hipLaunchKernelGGL((k_entry_fwd<TX, 12>), dim3(blocks), dim3(kEntBlock), 0, st, d, cp, idx, x, B,
                                    resid, part); break;
        default: hipLaunchKernelGGL((k_entry_fwd<TX, 16>), dim3(blocks), dim3(kEntBlock), 0, st, d, cp, idx, x, B,
                                    resid, part); break;
    }
}

static void launch_entry_bwd(const tr_desc& d, const EntryPlan& P, Ptrs cp, const int32_t* idx, const float* resid,
                             int B, float scale, const double* scale_dev, float* gpart, float* red, MutPtrs grads,
                             hipStream_t st) {
#define TRK_BWD(LDS, RMV)                                                                                         \
    hipLaunchKernelGGL((k_entry_bwd_acc<LDS, RMV>), dim3(P.bwd_blocks), dim3(P.bwd_threads), P.bwd_shm, st, d, cp, \
                       idx, resid, B, P.EPB, P.SB, P.PF, scale, scale_dev, gpart, P.slice_len)
    const int rm = rank_bound(d);
    if (P.slice_lds) {
        if (rm == 4) TRK_BWD(true, 4);
        else if (rm == 8) TRK_BWD(true, 8);
        else if (rm == 12) TRK_BWD(true, 12);
        else TRK_BWD(true, 16);
    } else {
        if (rm == 4) TRK_BWD(false, 4);
        else if (rm == 8) TRK_BWD(false, 8);
        else if (rm == 12) TRK_BWD(false, 12);
        else TRK_BWD(false, 16);
    }
#undef TRK_BWD
    const unsigned eb = (unsigned)((P.slice_len + 255) / 256);
    hipLaunchKernelGGL(k_entry_bwd_reduce1, dim3(eb, (unsigned)P.QG), dim3(256), 0, st, gpart, P.bwd_blocks, P.QG,
                       P.slice_len, red);
    hipLaunchKernelGGL(k_entry_bwd_reduce2, dim3(eb), dim3(256), 0, st, d, red, P.QG, P.slice_len, grads);
}

struct CompletionWs {
    EntryPlan P;
    size_t bidx, bx, resid, grads, loss, total;
};

static CompletionWs completion_layout(const tr_desc& d, int B) {
    CompletionWs L{};
    L.P = entry_plan(d, B);
    size_t o = align_up(L.P.total);
    L.bidx = o;
    o += align_up((size_t)B * d.N * 4);
    L.bx = o;
    o += align_up((size_t)B * 4);
    L.resid = o;
    o += align_up((size_t)B * 4);
    L.grads = o;
    o += align_up((size_t)L.P.slice_len * 4);
    L.loss = o;
    o += align_up(8);
    L.total = o;
    return L;
}

}  // namespace trk

using namespace trk;

extern "C" {

size_t tr_entry_workspace_size(const tr_desc* d, int32_t B) {
    if (validate_desc(d) != TR_OK || B < 1) return 0;
    return entry_plan(*d, B).total;
}

static tr_status entry_checks(const tr_desc* d, const void* const* cores, const int32_t* idx, int32_t B) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (d->core_dtype != TR_F32) return TR_E_DTYPE;
    if (!cores || !idx) return TR_E_ARG;
    for (int k = 0; k < d->N; ++k)
        if (!cores[k]) return TR_E_ARG;
    if (B < 1 || B > (1 << 26)) return TR_E_SHAPE;
    return TR_OK;
}

tr_status tr_entry_fwd(const tr_desc* d, const void* const* cores, const int32_t* idx, const void* x, int32_t B,
                       float* resid, double* loss, void* ws, size_t ws_bytes, tr_stream_t stream) {
    tr_status s = entry_checks(d, cores, idx, B);
    if (s != TR_OK) return s;
    if (!x || !resid) return TR_E_ARG;
    const EntryPlan P = entry_plan(*d, B);
    if (!ws || ws_bytes < P.total) return TR_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Ptrs cp{};
    for (int k = 0; k < d->N; ++k) cp.p[k] = cores[k];
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + P.part_off);
    switch (d->x_dtype) {
        case TR_F32:
            launch_entry_fwd(*d, cp, idx, static_cast<const float*>(x), B, resid, part, P.fwd_blocks, st);
            break;
        case TR_F16:
            launch_entry_fwd(*d, cp, idx, static_cast<const __half*>(x), B, resid, part, P.fwd_blocks, st);
            break;
        default:
            return TR_E_DTYPE;
    }
    if (hipGetLastError() != hipSuccess) return TR_E_HIP;
    if (loss) {
        hipLaunchKernelGGL(k_entry_loss, dim3(1), dim3(256), 0, st, part, P.fwd_blocks, B, loss);
        if (hipGetLastError() != hipSuccess) return TR_E_HIP;
    }
    return TR_OK;
}

tr_status tr_entry_bwd(const tr_desc* d, const void* const* cores, const int32_t* idx, const float* resid, int32_t B,
                       double scale, const double* scale_dev, void* const* grads, void* ws, size_t ws_bytes,
                       tr_stream_t stream) {
    tr_status s = entry_checks(d, cores, idx, B);
    if (s != TR_OK) return s;
    if (!resid || !grads) return TR_E_ARG;
    for (int k = 0; k < d->N; ++k)
        if (!grads[k]) return TR_E_ARG;
    const EntryPlan P = entry_plan(*d, B);
    if (!ws || ws_bytes < P.total) return TR_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Ptrs cp{};
    MutPtrs gp{};
    for (int k = 0; k < d->N; ++k) {
        cp.p[k] = cores[k];
        gp.p[k] = grads[k];
    }
    char* w = static_cast<char*>(ws);
    launch_entry_bwd(*d, P, cp, idx, resid, B, (float)scale, scale_dev, reinterpret_cast<float*>(w + P.gpart_off),
                     reinterpret_cast<float*>(w + P.red_off), gp, st);
    return hipGetLastError() == hipSuccess ? TR_OK : TR_E_HIP;
}

static tr_status completion_checks(const tr_desc* d, const tr_completion_config* c) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (!c) return TR_E_ARG;
    if (d->core_dtype != TR_F32) return TR_E_DTYPE;
    if (d->x_dtype != TR_F32 && d->x_dtype != TR_F16) return TR_E_DTYPE;
    if (c->B < 1 || c->B > (1 << 26)) return TR_E_SHAPE;
    if (!(c->lambda >= 0.0)) return TR_E_ARG;
    if (c->rule.kind < 0 || c->rule.kind > 2) return TR_E_ARG;
    if (c->rule.kind == 2 && !(c->rule.tau > 0.0)) return TR_E_ARG;
    return TR_OK;
}

size_t tr_completion_workspace_size(const tr_desc* d, const tr_completion_config* c) {
    if (completion_checks(d, c) != TR_OK) return 0;
    return completion_layout(*d, c->B).total;
}

tr_status tr_completion_run(const tr_desc* d, void* const* cores, void* const* accum, const int32_t* obs_idx,
                            const void* obs_x, int64_t n_obs, const tr_completion_config* c, uint64_t* t_dev,
                            int32_t steps, double* loss_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                            tr_stream_t stream) {
    tr_status s = completion_checks(d, c);
    if (s != TR_OK) return s;
    if (!cores || !obs_idx || !obs_x || !t_dev || n_obs < 1 || steps < 0) return TR_E_ARG;
    for (int k = 0; k < d->N; ++k) {
        if (!cores[k]) return TR_E_ARG;
        if (c->rule.kind == 1 && (!accum || !accum[k])) return TR_E_ARG;
    }
    const CompletionWs L = completion_layout(*d, c->B);
    if (!ws || ws_bytes < L.total) return TR_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return TR_E_ALIGN;
    if (steps == 0) return TR_OK;
    hipStream_t st = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    double* part = reinterpret_cast<double*>(w + L.P.part_off);
    float* gpart = reinterpret_cast<float*>(w + L.P.gpart_off);
    float* red = reinterpret_cast<float*>(w + L.P.red_off);
    int32_t* bidx = reinterpret_cast<int32_t*>(w + L.bidx);
    float* resid = reinterpret_cast<float*>(w + L.resid);
    float* grads = reinterpret_cast<float*>(w + L.grads);
    double* lossw = reinterpret_cast<double*>(w + L.loss);
    Ptrs cp{};
    MutPtrs mc{}, ac{}, gp{};
    int64_t off = 0;
    for (int k = 0; k < d->N; ++k) {
        cp.p[k] = cores[k];
        mc.p[k] = cores[k];
        ac.p[k] = accum ? accum[k] : nullptr;
        gp.p[k] = grads + off;
        off += (int64_t)d->I[k] * d->R[k] * d->R[ring_next(k, d->N)];
    }
    const int B = c->B;
    const dim3 gd((unsigned)((B + 255) / 256));
    const dim3 gu((unsigned)((L.P.slice_len + 255) / 256));
    for (int it = 0; it < steps; ++it) {
        double* loss = loss_out ? loss_out + it : lossw;
        if (d->x_dtype == TR_F32) {
            float* bx = reinterpret_cast<float*>(w + L.bx);
            hipLaunchKernelGGL(k_completion_draw<float>, gd, dim3(256), 0, st, *d, t_dev, c->seed, obs_idx,
                               static_cast<const float*>(obs_x), n_obs, B, bidx, bx);
            launch_entry_fwd(*d, cp, bidx, static_cast<const float*>(bx), B, resid, part, L.P.fwd_blocks, st);
        } else {
            __half* bx = reinterpret_cast<__half*>(w + L.bx);
            hipLaunchKernelGGL(k_completion_draw<__half>, gd, dim3(256), 0, st, *d, t_dev, c->seed, obs_idx,
                               static_cast<const __half*>(obs_x), n_obs, B, bidx, bx);
            launch_entry_fwd(*d, cp, bidx, static_cast<const __half*>(bx), B, resid, part, L.P.fwd_blocks, st);
        }
        hipLaunchKernelGGL(k_completion_loss, dim3(1), dim3(256), 0, st, *d, part, L.P.fwd_blocks, B, cp, c->lambda,
                           loss);
        launch_entry_bwd(*d, L.P, cp, bidx, resid, B, 1.0f, nullptr, gpart, red, gp, st);
        hipLaunchKernelGGL(k_completion_update, gu, dim3(256), 0, st, *d, t_dev, c->seed, (int)c->block, mc, ac,
                           grads, L.P.slice_len, c->lambda, c->rule, dev_status);
        if (hipGetLastError() != hipSuccess) return TR_E_HIP;
        if (launch_bump(t_dev, st) != hipSuccess) return TR_E_HIP;
    }
    return TR_OK;
}

}  // extern "C"
