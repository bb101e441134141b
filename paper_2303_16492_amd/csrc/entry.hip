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
// the workspace, each (k, column) owned by one thread; a second kernel adds
// the block slices in a fixed order.  No float atomics: results are bitwise
// reproducible.
#include "internal.hpp"

namespace trk {

constexpr int kEntBlock = 256;

// Row ``s`` of A_{k0} A_{k0+1} ... (``len`` slices cyclically from k0) for entry idx.
__device__ inline void chain_row(const tr_desc& d, const Ptrs& cores, const int32_t* ik, int k0, int len, int s,
                                 float* v) {
    const int N = d.N;
    int k = k0;
    {
        const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
        const float* A = static_cast<const float*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
#pragma unroll
        for (int c = 0; c < kMaxRank; ++c) v[c] = c < Rk1 ? A[s + Rk * c] : 0.f;
    }
    for (int q = 1; q < len; ++q) {
        k = ring_next(k, N);
        const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
        const float* A = static_cast<const float*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
        float w[kMaxRank];
#pragma unroll
        for (int c = 0; c < kMaxRank; ++c) {
            float acc = 0.f;
            if (c < Rk1) {
#pragma unroll
                for (int r = 0; r < kMaxRank; ++r)
                    if (r < Rk) acc += v[r] * A[r + Rk * c];
            }
            w[c] = acc;
        }
#pragma unroll
        for (int c = 0; c < kMaxRank; ++c) v[c] = w[c];
    }
}

template <typename TX>
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
            float v[kMaxRank];
            chain_row(d, cores, ik, 0, N, s, v);
#pragma unroll
            for (int c = 0; c < kMaxRank; ++c)
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

__global__ void k_entry_loss(const double* __restrict__ part, int nb, int B, double* loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < nb; ++q) s += part[q];
    *loss = s / (2.0 * (double)B);
}

// Backward, phase 1: per block of EPB entries, ordered accumulation into the
// block's private gradient slice gpart[block][sum_k I_k RR_k].
__global__ __launch_bounds__(kEntBlock) void k_entry_bwd_acc(tr_desc d, Ptrs cores, const int32_t* __restrict__ idx,
                                                             const float* __restrict__ resid, int B, int EPB, int SB,
                                                             float scale, const double* __restrict__ dscale,
                                                             float* __restrict__ gpart, int64_t slice_len) {
    const int N = d.N;
    int rowsum = 0, ccount = 0;       // rows of all M_{!=k}, total columns
    int64_t gofs[kMaxOrder];
    int cofs[kMaxOrder], rofs[kMaxOrder];
    {
        int64_t go = 0;
        for (int k = 0; k < N; ++k) {
            const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
            rofs[k] = rowsum;
            cofs[k] = ccount;
            gofs[k] = go;
            rowsum += Rk1;
            ccount += Rk * Rk1;
            go += (int64_t)d.I[k] * Rk * Rk1;
        }
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* cb = reinterpret_cast<float*>(smem_raw);                  // [SB][ccount]
    int* sidx = reinterpret_cast<int*>(cb + (size_t)SB * ccount);     // [SB][N]
    float* sres = reinterpret_cast<float*>(sidx + SB * N);            // [SB]
    float* G = gpart + (int64_t)blockIdx.x * slice_len;
    for (int64_t e = threadIdx.x; e < slice_len; e += blockDim.x) G[e] = 0.f;
    // dL/dG_k of L = 1/(2B) sum r^2: the 1/B of the mean applied here
    const float sc = (float)((double)scale * (dscale ? *dscale : 1.0) / (double)B);
    const int64_t b0 = (int64_t)blockIdx.x * EPB;
    const int64_t b1 = min((int64_t)B, b0 + EPB);
    for (int64_t bs = b0; bs < b1; bs += SB) {
        const int nb = (int)min((int64_t)SB, b1 - bs);
        __syncthreads();
        for (int e = threadIdx.x; e < nb * N; e += blockDim.x) {
            const int k = e % N, v = idx[bs * N + e];
            sidx[e] = (v >= 0 && v < d.I[k]) ? v : -1;   // -1: invalid caller index, entry skipped
        }
        for (int e = threadIdx.x; e < nb; e += blockDim.x) sres[e] = resid[bs + e] * sc;
        __syncthreads();
        // contributions: thread per (entry, k, row s of M_{!=k})
        for (int e = threadIdx.x; e < nb * rowsum; e += blockDim.x) {
            const int lb = e / rowsum, rr = e % rowsum;
            bool ok = true;
            for (int q = 0; q < N; ++q) ok = ok && sidx[lb * N + q] >= 0;
            if (!ok) continue;
            int k = 0;
            while (k + 1 < N && rofs[k + 1] <= rr) ++k;
            const int s = rr - rofs[k];
            const int Rk = d.R[k];
            float v[kMaxRank];
            chain_row(d, cores, sidx + lb * N, ring_next(k, N), N - 1, s, v);
            float* out = cb + (size_t)lb * ccount + cofs[k] + Rk * s;
            const float rv = sres[lb];
#pragma unroll
            for (int r = 0; r < kMaxRank; ++r)
                if (r < Rk) out[r] = rv * v[r];
        }
        __syncthreads();
        // ordered accumulation: thread owns columns (k, c)
        for (int lb = 0; lb < nb; ++lb) {
            for (int p = threadIdx.x; p < ccount; p += blockDim.x) {
                int k = 0;
                while (k + 1 < N && cofs[k + 1] <= p) ++k;
                const int c = p - cofs[k];
                const int RRk = d.R[k] * d.R[ring_next(k, N)];
                bool ok = true;
                for (int q = 0; q < N; ++q) ok = ok && sidx[lb * N + q] >= 0;
                if (!ok) continue;
                const int i = sidx[lb * N + k];
                G[gofs[k] + (int64_t)i * RRk + c] += cb[(size_t)lb * ccount + p];
            }
        }
    }
}

// Backward, phase 2: grads[k][e] = sum over blocks (fixed order).
__global__ __launch_bounds__(256) void k_entry_bwd_reduce(tr_desc d, const float* __restrict__ gpart, int nblocks,
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
    for (int q = 0; q < nblocks; ++q) s += gpart[(int64_t)q * slice_len + e];
    static_cast<float*>(grads.p[k])[e - base] = s;
}

struct EntryPlan {
    int fwd_blocks, bwd_blocks, EPB, SB;
    int64_t slice_len;
    size_t part_off, gpart_off, total, bwd_shm;
};

static EntryPlan entry_plan(const tr_desc& d, int B) {
    EntryPlan P{};
    const int per = kEntBlock / d.R[0];
    P.fwd_blocks = (B + per - 1) / per;
    int ccount = 0;
    int64_t sl = 0;
    for (int k = 0; k < d.N; ++k) {
        const int rr = d.R[k] * d.R[ring_next(k, d.N)];
        ccount += rr;
        sl += (int64_t)d.I[k] * rr;
    }
    P.slice_len = sl;
    P.EPB = 128;
    P.bwd_blocks = (B + P.EPB - 1) / P.EPB;
    int SB = 32;
    while (SB > 1 && (size_t)SB * (ccount * 4 + d.N * 4 + 4) > 48 * 1024) SB >>= 1;
    P.SB = SB;
    P.bwd_shm = (size_t)SB * ccount * 4 + (size_t)SB * d.N * 4 + SB * 4 + 64;
    P.part_off = 0;
    P.gpart_off = align_up((size_t)P.fwd_blocks * 8);
    P.total = P.gpart_off + align_up((size_t)P.bwd_blocks * sl * 4);
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
// lambda/2 sum_k ||G_k||^2 (strided per thread, then the block tree).
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
    if (threadIdx.x == 0) {
        double data = 0.0;
        for (int q = 0; q < nb; ++q) data += part[q];
        *loss = data / (2.0 * (double)B) + 0.5 * lam * ridge;
    }
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
            hipLaunchKernelGGL(k_entry_fwd<float>, dim3(P.fwd_blocks), dim3(kEntBlock), 0, st, *d, cp, idx,
                               static_cast<const float*>(x), B, resid, part);
            break;
        case TR_F16:
            hipLaunchKernelGGL(k_entry_fwd<__half>, dim3(P.fwd_blocks), dim3(kEntBlock), 0, st, *d, cp, idx,
                               static_cast<const __half*>(x), B, resid, part);
            break;
        default:
            return TR_E_DTYPE;
    }
    if (hipGetLastError() != hipSuccess) return TR_E_HIP;
    if (loss) {
        hipLaunchKernelGGL(k_entry_loss, dim3(1), dim3(64), 0, st, part, P.fwd_blocks, B, loss);
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
    float* gpart = reinterpret_cast<float*>(static_cast<char*>(ws) + P.gpart_off);
    hipLaunchKernelGGL(k_entry_bwd_acc, dim3(P.bwd_blocks), dim3(kEntBlock), P.bwd_shm, st, *d, cp, idx, resid, B,
                       P.EPB, P.SB, (float)scale, scale_dev, gpart, P.slice_len);
    if (hipGetLastError() != hipSuccess) return TR_E_HIP;
    hipLaunchKernelGGL(k_entry_bwd_reduce, dim3((unsigned)((P.slice_len + 255) / 256)), dim3(256), 0, st, *d, gpart,
                       P.bwd_blocks, P.slice_len, gp);
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
            hipLaunchKernelGGL(k_entry_fwd<float>, dim3(L.P.fwd_blocks), dim3(kEntBlock), 0, st, *d, cp, bidx, bx, B,
                               resid, part);
        } else {
            __half* bx = reinterpret_cast<__half*>(w + L.bx);
            hipLaunchKernelGGL(k_completion_draw<__half>, gd, dim3(256), 0, st, *d, t_dev, c->seed, obs_idx,
                               static_cast<const __half*>(obs_x), n_obs, B, bidx, bx);
            hipLaunchKernelGGL(k_entry_fwd<__half>, dim3(L.P.fwd_blocks), dim3(kEntBlock), 0, st, *d, cp, bidx, bx,
                               B, resid, part);
        }
        hipLaunchKernelGGL(k_completion_loss, dim3(1), dim3(256), 0, st, *d, part, L.P.fwd_blocks, B, cp, c->lambda,
                           loss);
        hipLaunchKernelGGL(k_entry_bwd_acc, dim3(L.P.bwd_blocks), dim3(kEntBlock), L.P.bwd_shm, st, *d, cp, bidx,
                           resid, B, L.P.EPB, L.P.SB, 1.0f, nullptr, gpart, L.P.slice_len);
        hipLaunchKernelGGL(k_entry_bwd_reduce, dim3((unsigned)((L.P.slice_len + 255) / 256)), dim3(256), 0, st, *d,
                           gpart, L.P.bwd_blocks, L.P.slice_len, gp);
        hipLaunchKernelGGL(k_completion_update, gu, dim3(256), 0, st, *d, t_dev, c->seed, (int)c->block, mc, ac,
                           grads, L.P.slice_len, c->lambda, c->rule, dev_status);
        if (hipGetLastError() != hipSuccess) return TR_E_HIP;
        if (launch_bump(t_dev, st) != hipSuccess) return TR_E_HIP;
    }
    return TR_OK;
}

}  // extern "C"
