// a5/a6 (+ the Gram of a7): fiber gather, stochastic gradient, loss estimate.
//
// g = (G_{n(2)} S^T D S - X_F D S) / (m J_n) (equation eq:S_gradient) is
// evaluated prediction-first: E = X_F - G_{n(2)} S^T, then g = -E D S/(m J_n).
// The Gram-first order of the paper's cost remark subtracts two large terms
// and, multiplied by an ill-conditioned inverse Gram in the scaled variant,
// loses every digit; prediction-first keeps the error relative to E.
//
// Work split: blocks tile (rows of G_{n(2)}) x (groups of sample chunks).
// A block gathers the X_F tile straight from HBM (one fiber per sample,
// contiguous when a mode-major replica is given), forms E in LDS and keeps
// its g rows in registers across its chunks; partial sums per group go to
// the workspace and are added in a fixed order by the reduce kernel, so
// results are bitwise reproducible.
#include "internal.hpp"

namespace trk {

namespace {

template <typename TC>
struct GradCfg;
template <> struct GradCfg<double> { static constexpr int TI = 32, TF = 32; };

__device__ inline void fiber_strides(const tr_desc& d, int n, bool replica, int64_t* xs) {
    if (!replica) {
        for (int k = 0; k < d.N; ++k) xs[k] = d.x_stride[k];
        return;
    }
    int64_t s = d.I[n];
    xs[n] = 1;
    int k = n;
    for (int q = 1; q < d.N; ++q) {
        k = ring_next(k, d.N);
        xs[k] = s;
        s *= d.I[k];
    }
}

}  // namespace

template <typename TC, typename TX>
__global__ __launch_bounds__(256) void k_grad_partial(tr_desc d, ModeSrc ms, Ptrs cores, XSrc xsrc,
                                                      const int32_t* __restrict__ idx,
                                                      const TC* __restrict__ S,
                                                      const double* __restrict__ pF, int m,
                                                      int groups, int row_tiles_max, int RRp,
                                                      TC* __restrict__ gpart,
                                                      double* __restrict__ lpart, int maxIRR) {
    int rtile, grp;
    if (!xcd_tile_group(row_tiles_max, groups, rtile, grp)) return;
    constexpr int TI = GradCfg<TC>::TI, TF = GradCfg<TC>::TF;
    constexpr int MAXO = TI * kMaxRR / 256;
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int N = d.N;
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, N)];
    const int i0 = rtile * TI;
    if (i0 >= In) return;
    const int tid = threadIdx.x;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    TC* sS = reinterpret_cast<TC*>(smem_raw);       // [TF][RRp]
    TC* sG = sS + TF * RRp;                         // [TI][RRp]
    TC* sE = sG + TI * RRp;                         // [TI][TF+1]
    TC* sW = sE + TI * (TF + 1);                    // [TF]
    double* sL = reinterpret_cast<double*>(sW + TF + (TF & 1));   // [TF]
    int64_t* sB = reinterpret_cast<int64_t*>(sL + TF);            // [TF]

    const TC* Gn = static_cast<const TC*>(cores.p[n]);
    for (int e = tid; e < TI * RRp; e += 256) {
        const int i = e / RRp, c = e - (e / RRp) * RRp;
        sG[e] = (i0 + i < In && c < RR) ? Gn[(int64_t)(i0 + i) * RR + c] : TC(0);
    }
    const bool rep = xsrc.rep[n] != nullptr;
    const TX* X = static_cast<const TX*>(rep ? xsrc.rep[n] : xsrc.X);
    int64_t xs[kMaxOrder];
    fiber_strides(d, n, rep, xs);
    const int64_t xsn = xs[n];

    TC acc[MAXO];
#pragma unroll
    for (int q = 0; q < MAXO; ++q) acc[q] = TC(0);
    double lsum = 0.0;
    const double Jn = (double)J_of(d, n);
    const double wbase = 1.0 / ((double)m * Jn);

    const int nchunks = (m + TF - 1) / TF;
    const int cpg = (nchunks + groups - 1) / groups;
    const int cbeg = grp * cpg, cend = min(nchunks, cbeg + cpg);
    for (int ch = cbeg; ch < cend; ++ch) {
        const int f0 = ch * TF;
        __syncthreads();
        for (int e = tid; e < TF * RRp; e += 256) {
            const int f = e / RRp, c = e - (e / RRp) * RRp;
            sS[e] = (f0 + f < m && c < RR) ? S[(int64_t)(f0 + f) * RR + c] : TC(0);
        }
        if (tid < TF) {
            const int f = f0 + tid;
            bool ok = f < m;
            int64_t off = 0;
            if (ok) {
                for (int k = 0; k < N; ++k) {
                    if (k == n) continue;
                    const int ik = idx[(int64_t)f * N + k];
                    if (ik < 0 || ik >= d.I[k]) ok = false;
                    off += (int64_t)ik * xs[k];
                }
            }
            if (ok) {
                sB[tid] = off;
                sW[tid] = (TC)(wbase / pF[f]);
                sL[tid] = 1.0 / (2.0 * (double)m * pF[f]);
            } else {   // past the end, or an invalid caller index: contributes nothing
                sB[tid] = 0;
                sW[tid] = TC(0);
                sL[tid] = 0.0;
            }
        }
        __syncthreads();
        // E = X_F - G S^T for the tile, scaled by -w_f into sE.
        for (int o = tid; o < TI * TF; o += 256) {
            const int i = o % TI, f = o / TI;
            TC val = TC(0);
            if (i0 + i < In && f0 + f < m && sW[f] != TC(0)) {
                TC dot = TC(0);
                const TC* gr = sG + i * RRp;
                const TC* sr = sS + f * RRp;
                for (int c = 0; c < RR; ++c) dot += gr[c] * sr[c];
                const TC x = (TC)to_f64(X[sB[f] + (int64_t)(i0 + i) * xsn]);
                const TC e = x - dot;
                lsum += (double)e * (double)e * sL[f];
                val = -e * sW[f];
            }
            sE[i * (TF + 1) + f] = val;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MAXO; ++q) {
            const int o = tid + 256 * q;
            if (o < TI * RR) {
                const int i = o / RR, c = o - (o / RR) * RR;
                const TC* er = sE + i * (TF + 1);
                TC a = acc[q];
                for (int f = 0; f < TF; ++f) a += er[f] * sS[f * RRp + c];
                acc[q] = a;
            }
        }
    }
    TC* out = gpart + (int64_t)grp * maxIRR;
#pragma unroll
    for (int q = 0; q < MAXO; ++q) {
        const int o = tid + 256 * q;
        if (o < TI * RR) {
            const int i = o / RR, c = o - (o / RR) * RR;
            if (i0 + i < In) out[(int64_t)(i0 + i) * RR + c] = acc[q];
        }
    }
    __shared__ double red[4];
    const double tot = block_sum(lsum, red);
    if (tid == 0) lpart[(int64_t)grp * row_tiles_max + rtile] = tot;
}

// Fixed-order sum of the partials; optional plain update G += rule(-g).
template <typename TC>
__global__ __launch_bounds__(256) void k_grad_reduce(tr_desc d, ModeSrc ms, const TC* __restrict__ gpart,
                                                     const double* __restrict__ lpart, int groups,
                                                     int row_tiles_max, int TI, int maxIRR,
                                                     TC* __restrict__ g, double* __restrict__ loss,
                                                     int apply, MutPtrs cores, MutPtrs accum,
                                                     tr_step rule, int32_t* status, StepBump step) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    const int64_t total = (int64_t)In * RR;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && loss) {
        __shared__ double red[4];
        const double s = loss_parts_sum(LossParts{lpart, groups, row_tiles_max, TI}, In, red);
        if (threadIdx.x == 0) *loss = s;
    }
    if (e < total) {
        constexpr int GB = 32;   // partial slices fetched together, added in group order
        TC acc = TC(0);
        for (int gi = 0; gi < groups; gi += GB) {
            TC v[GB];
#pragma unroll
            for (int u = 0; u < GB; ++u) v[u] = gi + u < groups ? gpart[(int64_t)(gi + u) * maxIRR + e] : TC(0);
#pragma unroll
            for (int u = 0; u < GB; ++u)
                if (gi + u < groups) acc += v[u];
        }
        if (g) g[e] = acc;
        if (apply) {
            TC* G = static_cast<TC*>(cores.p[n]);
            TC* A = static_cast<TC*>(accum.p[n]);
            apply_rule<TC>(G, A, e, -(double)acc, rule, t, status);
        }
    }
    bump_if_last(step, rule.kind == 2);
}

GradWs grad_ws_layout(const tr_desc& d, int m, int prec) {
    GradWs L{};
    const Shape sh = shape_of(d);
    const bool f64 = d.core_dtype == TR_F64;
    L.ti = f64 ? GradCfg<double>::TI : 64;   // FP32 runs the matrix-core kernel (64-row tiles)
    L.tf = f64 ? GradCfg<double>::TF : 64;
    L.row_tiles = (sh.maxI + L.ti - 1) / L.ti;
    // about one block per CU (two for FP64): fewer partial slices to add
    // afterwards.  With the XCD-aware order (a group's row tiles on one XCD
    // of 32 CUs) a multiple of 8 groups with at most that many blocks per
    // XCD, so that no XCD takes a second round of blocks.
    const int per_xcd = f64 ? 64 : 32;
    int groups = ((f64 ? 512 : 256) + L.row_tiles - 1) / L.row_tiles;
    if (L.row_tiles <= per_xcd && groups >= 8) groups = 8 * (per_xcd / L.row_tiles);
    // FP32 with R_n R_{n+1} <= 128: chunks of 128 samples when that still
    // gives at least half of those blocks
    if (!f64 && sh.maxRR <= 128 && 2 * ((m + 127) / 128) >= groups) L.tf = 128;
    const int nchunks = (m + L.tf - 1) / L.tf;
    groups = groups < 1 ? 1 : groups;
    groups = groups > nchunks ? nchunks : groups;
    const int cpg = (nchunks + groups - 1) / groups;
    L.groups = (nchunks + cpg - 1) / cpg;
    if (L.groups < 1) L.groups = 1;
    const size_t es = f64 ? 8 : 4;
    L.gpart_off = 0;
    L.lpart_off = align_up((size_t)L.groups * sh.maxI * sh.maxRR * es);
    L.total = L.lpart_off + align_up((size_t)L.groups * L.row_tiles * 8);
    (void)prec;
    return L;
}

hipError_t launch_grad_partial(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx,
                               const void* S, const double* pF, int m, int prec, void* ws,
                               const GradWs& L, hipStream_t st) {
    const Shape sh = shape_of(d);
    const int RRp = sh.maxRR | 1;   // odd row pitch: rows of sG/sS fall in different LDS banks
    const dim3 grid(xcd_grid(L.row_tiles, L.groups));
    char* w = static_cast<char*>(ws);
    const int maxIRR = sh.maxI * sh.maxRR;
    if (d.core_dtype == TR_F64) {
        constexpr int TI = GradCfg<double>::TI, TF = GradCfg<double>::TF;
        const size_t shm = (size_t)(TF * RRp + TI * RRp + TI * (TF + 1) + TF + 1) * 8 + TF * 16;
        if (d.x_dtype != TR_F64) return hipErrorInvalidValue;
        if (!allow_lds(reinterpret_cast<const void*>(&k_grad_partial<double, double>), shm)) return hipErrorInvalidValue;
        launch_timed(k_grad_partial<double, double>, grid, dim3(256), shm, st, d, ms, cores, xs, idx,
                     static_cast<const double*>(S), pF, m, L.groups, L.row_tiles, RRp,
                     reinterpret_cast<double*>(w + L.gpart_off), reinterpret_cast<double*>(w + L.lpart_off),
                     maxIRR);
    } else if (prec == TR_PREC_BF16 || prec == TR_PREC_F16) {
        return launch_grad_mixed(d, ms, cores, xs, idx, static_cast<const float*>(S), pF, m, prec, L.groups,
                                 L.row_tiles, reinterpret_cast<float*>(w + L.gpart_off),
                                 reinterpret_cast<double*>(w + L.lpart_off), st);
    } else {
        return launch_grad_mfma_f32(d, ms, cores, xs, idx, static_cast<const float*>(S), pF, m, L.groups, L.row_tiles,
                                    reinterpret_cast<float*>(w + L.gpart_off), reinterpret_cast<double*>(w + L.lpart_off),
                                    L.tf, st);
    }
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const tr_desc& d, ModeSrc ms, const void* ws, const GradWs& L, void* g,
                              double* loss, bool apply, MutPtrs cores, MutPtrs accum, tr_step rule,
                              int32_t* status, hipStream_t st, StepBump step) {
    const Shape sh = shape_of(d);
    const int maxIRR = sh.maxI * sh.maxRR;
    const dim3 grid((unsigned)((maxIRR + 255) / 256));
    const char* w = static_cast<const char*>(ws);
    const double* lp = reinterpret_cast<const double*>(w + L.lpart_off);
    if (d.core_dtype == TR_F64)
        hipLaunchKernelGGL(k_grad_reduce<double>, grid, dim3(256), 0, st, d, ms,
                           reinterpret_cast<const double*>(w + L.gpart_off), lp, L.groups, L.row_tiles,
                           L.ti, maxIRR, static_cast<double*>(g), loss, (int)apply, cores, accum, rule,
                           status, step);
    else
        hipLaunchKernelGGL(k_grad_reduce<float>, grid, dim3(256), 0, st, d, ms,
                           reinterpret_cast<const float*>(w + L.gpart_off), lp, L.groups, L.row_tiles,
                           L.ti, maxIRR, static_cast<float*>(g), loss, (int)apply, cores, accum, rule,
                           status, step);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Gram --
// gram[c][c'] = sum_f S[f][c] S[f][c'] / (m J_n pF_f), products and sums in
// FP64 from the stored S.  Blocks take the lower-triangular 32 x 32 tiles
// of the RR x RR output times groups of samples (the tiles of one group on
// one XCD, so the group's rows of S come from that XCD's L2 after the first
// tile fetched them): a block fetches its
// samples' S columns and weights in one batch (FP32 S stays FP32 in LDS),
// then each wavefront accumulates one 16 x 16 quadrant of the tile on the
// FP64 matrix cores.  A second kernel adds the
// groups in a fixed order and mirrors the lower triangle.

constexpr int kGramT = 32;
template <typename TC>
struct GramChunk {   // samples staged per round: 2 x F x 33 values of TC stay under 64 KiB
    // (FP32: 192, so a group of m / 24 samples at m = 4096 is one round, all
    // of its loads in flight together)
    static constexpr int F = sizeof(TC) == 8 ? 64 : 192;
};

__host__ __device__ inline void gram_tile(int tile, int& ct, int& et) {   // tile -> (ct >= et)
    ct = 0;
    while ((ct + 1) * (ct + 2) / 2 <= tile) ++ct;
    et = tile - ct * (ct + 1) / 2;
}

template <typename TC>
__global__ __launch_bounds__(256) void k_gram_partial(tr_desc d, ModeSrc ms, const TC* __restrict__ S,
                                                      const double* __restrict__ pF, int m, int groups,
                                                      int tiles_max, double* __restrict__ part,
                                                      int maxRR2, Ptrs rows) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    // S null: the rows are those of G_{n(2)} itself (I_n of them), unweighted
    if (!S) {
        S = static_cast<const TC*>(rows.p[n]);
        m = d.I[n];
    }
    const int tpd = (RR + kGramT - 1) / kGramT;
    int tile, grp;
    if (!xcd_tile_group(tiles_max, groups, tile, grp)) return;
    if (tile >= tpd * (tpd + 1) / 2) return;
    int ct, et;
    gram_tile(tile, ct, et);
    const int c0 = ct * kGramT, e0 = et * kGramT;
    constexpr int kGramF = GramChunk<TC>::F;
    __shared__ TC sA[kGramF][kGramT + 1], sB[kGramF][kGramT + 1];
    __shared__ double sw[kGramF];
    const int tid = threadIdx.x;
    const double wbase = pF ? 1.0 / ((double)m * (double)J_of(d, n)) : 1.0;
    const int per = (m + groups - 1) / groups;
    const int fb = grp * per, fe = min(m, fb + per);
    // wavefront w computes the 16 x 16 quadrant (qr, qc) of the tile on the
    // FP64 matrix cores, K = 4 samples per instruction (lane l: A[l % 16][l / 16],
    // B[l / 16][l % 16], D[4 j + l / 16][l % 16])
    const int w = tid >> 6, l = tid & 63, lc = l & 15, lk = l >> 4;
    const int qr = w >> 1, qc = w & 1;
    typedef double gd4 __attribute__((ext_vector_type(4)));
    gd4 acc = {0.0, 0.0, 0.0, 0.0};
    // A round stages kGramF samples in two halves of rows: every load of
    // the round is issued first, the first half goes to LDS as soon as its
    // loads have landed, and its matrix-core steps run while the second
    // half's loads are still in flight (the halves are disjoint rows).
    constexpr int V = kGramF * kGramT / 256, VH = V / 2, FH = kGramF / 2;
    static_assert(V % 2 == 0 && FH % 4 == 0, "two halves of whole K steps");
    for (int f0 = fb; f0 < fe; f0 += kGramF) {
        __syncthreads();
        // loads at clamped (in-bounds) indices, masked afterwards: no load
        // sits behind a branch, so the first half's wait counts only the
        // loads issued before its own
        const int c = tid & (kGramT - 1), fo = tid >> 5;   // row fo + 8 v, column c
        const bool okA = c0 + c < RR, okB = e0 + c < RR;
        const int cA = okA ? c0 + c : RR - 1, cB = okB ? e0 + c : RR - 1;
        double pv = 1.0;
        if (pF) {   // uniform
            const int fp = f0 + (tid < kGramF ? tid : 0);
            pv = pF[fp < fe ? fp : fe - 1];
        }
        TC av[V], bv[V];
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // the first half's loads issue first
#pragma unroll
            for (int v = h * VH; v < (h + 1) * VH; ++v) {
                const int f = f0 + fo + 8 * v, fr = f < fe ? f : fe - 1;
                av[v] = S[(int64_t)fr * RR + cA];
                bv[v] = S[(int64_t)fr * RR + cB];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        const int nf = min(kGramF, fe - f0);   // rows past nf are staged as zeros with weight 0
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int v = h * VH; v < (h + 1) * VH; ++v) {   // rows fo + 8 v of half h
                const int f = fo + 8 * v;
                const bool okf = f0 + f < fe;
                sA[f][c] = okf && okA ? av[v] : TC(0);
                sB[f][c] = okf && okB ? bv[v] : TC(0);
            }
            if (h == 0 && tid < kGramF) sw[tid] = f0 + tid < fe ? wbase / pv : 0.0;
            __syncthreads();
            const int qe = min(nf, (h + 1) * FH);
            for (int q = h * FH; q < qe; q += 4) {
                const int f = q + lk;
                const double a = (double)sA[f][16 * qr + lc] * sw[f];
                const double b = (double)sB[f][16 * qc + lc];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
        }
    }
    double* out = part + (int64_t)grp * maxRR2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = c0 + 16 * qr + 4 * j + lk, e = e0 + 16 * qc + lc;
        if (c < RR && e < RR) out[(int64_t)c * RR + e] = acc[j];
    }
}

// gram = sum of the group partials in group order; entries above the
// diagonal come from their mirror (only lower tiles are computed).
__global__ void k_gram_reduce(tr_desc d, ModeSrc ms, const double* __restrict__ part, int groups, int maxRR2,
                              double* __restrict__ gram) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= RR * RR) return;
    const int r = e / RR, c = e - r * RR;
    const bool lower = (r / kGramT) >= (c / kGramT);   // tile computed as stored
    const int src = lower ? e : c * RR + r;
    constexpr int GB = 32;
    double s = 0.0;
    for (int g = 0; g < groups; g += GB) {
        double v[GB];
        const double* q = part + (int64_t)g * maxRR2 + src;
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            v[u] = g + u < groups ? *q : 0.0;
            q += maxRR2;
        }
#pragma unroll
        for (int u = 0; u < GB; ++u)
            if (g + u < groups) s += v[u];
    }
    gram[e] = s;
}

GramWs gram_ws_layout(const tr_desc& d, int m) {
    GramWs L{};
    const Shape sh = shape_of(d);
    const int tpd = (sh.maxRR + kGramT - 1) / kGramT;
    L.tiles = tpd * (tpd + 1) / 2;
    // at most one block per CU (256), so that every block runs in the first
    // and only round: with the XCD-aware order (a group's tiles on one XCD
    // of 32 CUs) a multiple of 8 groups with at most 32 blocks per XCD;
    // at least 16 samples per group
    int groups = L.tiles <= 32 ? 8 * (32 / L.tiles) : 256 / L.tiles;
    const int gmax = (m + 15) / 16;
    groups = groups > gmax ? gmax : groups;
    groups = groups < 1 ? 1 : groups;
    const int per = (m + groups - 1) / groups;
    L.groups = (m + per - 1) / per;
    if (L.groups < 1) L.groups = 1;
    L.part_off = 0;
    L.total = align_up((size_t)L.groups * sh.maxRR * sh.maxRR * 8);
    return L;
}

hipError_t launch_gram(const tr_desc& d, ModeSrc ms, const void* S, const double* pF, int m, double* gram,
                       void* ws, const GramWs& L, hipStream_t st, hipEvent_t mid, Ptrs rows) {
    const Shape sh = shape_of(d);
    const int maxRR2 = sh.maxRR * sh.maxRR;
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + L.part_off);
    const dim3 grid(xcd_grid(L.tiles, L.groups));
    if (d.core_dtype == TR_F64)
        hipLaunchKernelGGL(k_gram_partial<double>, grid, dim3(256), 0, st, d, ms,
                           static_cast<const double*>(S), pF, m, L.groups, L.tiles, part, maxRR2, rows);
    else
        hipLaunchKernelGGL(k_gram_partial<float>, grid, dim3(256), 0, st, d, ms,
                           static_cast<const float*>(S), pF, m, L.groups, L.tiles, part, maxRR2, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (mid && (e = hipEventRecord(mid, st)) != hipSuccess) return e;
    // one wavefront per block: the partials' reads spread over as many CUs
    // as there are blocks of 64 entries
    hipLaunchKernelGGL(k_gram_reduce, dim3((maxRR2 + 63) / 64), dim3(64), 0, st, d, ms, part, L.groups, maxRR2,
                       gram);
    return hipGetLastError();
}

}  // namespace trk
