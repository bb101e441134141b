// a7/a8 for RR <= 128: the scaled direction p = -g (h + eta I)^{-1}
// (equation eq:scaledsg_direction with the damped preconditioner of the
// remark that follows it), then the step rule.
//
// The RR x RR system is inverted once per step instead of being solved for
// every one of the I_n rows of g: a blocked symmetric sweep (Gauss-Jordan
// elimination on an SPD matrix, eight pivots per block) turns M = h + eta I
// into -M^{-1} in one workgroup, and a second, row-parallel kernel forms
// p = g (-M^{-1}) and applies the rule.  A sweep pivot block is the Schur
// complement of the blocks already swept, so it is positive definite exactly
// when the matching Cholesky pivots are positive: the same test triggers the
// same fallback ladder eta + 10^(k-10) tr(h)/RR, k = 0..6.
//
// The matrix lives in FP64 matrix-core accumulators: 16 x 16 tiles of the
// lower triangle spread over four wavefronts (one per SIMD), so each block
// step moves only the eight pivot rows through LDS.  With U~ the pivot
// columns minus the selector E and V~ = U~^T, one block step is the single
// rank-8 update
//     M <- M - U~ B V~ - 2 E E^T,    B = (M_PP)^{-1},
// which gives -B on the pivot block, B M_PQ on its rows, M_QP B on its
// columns and M_QQ - M_QP B M_PQ elsewhere: the classical sweep.  Every
// wavefront factors the 8 x 8 pivot block itself (Cholesky, its inverse,
// then B), so the only barrier per step publishes the next pivot rows.
#include "internal.hpp"

namespace trk {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kSweepWaves = 4;

// Lower 16 x 16 tiles (rt >= ct) of an NT x NT tiling.  Wavefront w owns
// tile columns w and 2W-1-w, which balances the triangle: for NT = 7 or 8
// every wavefront holds the same number of tiles.  Slot k of wavefront w
// holds tile (w + k, w) for k < n1, and tile (NT - TPW + k, 2W-1-w) for the
// last n2 slots; every coordinate is a compile-time constant.
template <int NT>
struct SweepTiles {
    static constexpr int W = kSweepWaves;
    static constexpr int NP = 16 * NT;
    static constexpr int n1(int w) { return NT - w > 0 ? NT - w : 0; }
    static constexpr int n2(int w) { return NT - (2 * W - 1 - w) > 0 ? NT - (2 * W - 1 - w) : 0; }
    static constexpr int max_count() {
        int m = 0;
        for (int w = 0; w < W; ++w) m = n1(w) + n2(w) > m ? n1(w) + n2(w) : m;
        return m;
    }
    static constexpr int TPW = max_count();
};

// Slot k of wavefront wv: tile (slot_rt, slot_ct), or no tile.
template <int NT>
__host__ __device__ constexpr bool slot_first(int wv, int k) { return k < SweepTiles<NT>::n1(wv); }
template <int NT>
__host__ __device__ constexpr bool slot_second(int wv, int k) {
    return !slot_first<NT>(wv, k) && k >= SweepTiles<NT>::TPW - SweepTiles<NT>::n2(wv);
}
template <int NT>
__host__ __device__ constexpr bool slot_ok(int wv, int k) { return slot_first<NT>(wv, k) || slot_second<NT>(wv, k); }
template <int NT>
__host__ __device__ constexpr int slot_rt(int wv, int k) {
    return slot_first<NT>(wv, k) ? wv + k : (slot_second<NT>(wv, k) ? NT - SweepTiles<NT>::TPW + k : 0);
}
template <int NT>
__host__ __device__ constexpr int slot_ct(int wv, int k) {
    return slot_first<NT>(wv, k) ? wv : (slot_second<NT>(wv, k) ? 2 * kSweepWaves - 1 - wv : 0);
}

__device__ __forceinline__ int tri8(int i) { return (i * (i + 1)) >> 1; }

// Pivot block of step q (rows 8q.., read from the published pivot rows,
// which carry -1 on the pivot diagonal): Cholesky factor L, then
// V = L^{-1} over it, column by column (column j of V needs rows of L from
// column j on only).  Lane 0 stores V packed by rows (tri8(i) + j) into Vw.
// Every wavefront runs this same code on the same LDS data, so every
// wavefront reaches the same verdict.  Returns false on a pivot that is not
// positive.
__device__ __forceinline__ bool pivot_chol_inv(const double* __restrict__ Vt, int NP, int q, double* Vw) {
    double L[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) L[i][j] = Vt[i * NP + 8 * q + j];
        L[i][i] = Vt[i * NP + 8 * q + i] + 1.0;
    }
    bool good = true;
    double r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const double dj = L[j][j];
        good = good && (dj > 0.0) && isfinite(dj);
        r[j] = rsqrt(dj);
#pragma unroll
        for (int i = j + 1; i < 8; ++i) L[i][j] *= r[j];
#pragma unroll
        for (int k = j + 1; k < 8; ++k)
#pragma unroll
            for (int i = k; i < 8; ++i) L[i][k] -= L[i][j] * L[k][j];
    }
    double (&V)[8][8] = L;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
        for (int i = j + 1; i < 8; ++i) {
            double s = L[i][j] * r[j];
#pragma unroll
            for (int k = j + 1; k < i; ++k) s += L[i][k] * V[k][j];
            V[i][j] = -r[i] * s;
        }
        V[j][j] = r[j];
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) Vw[tri8(i) + j] = V[i][j];
    }
    return good;
}

// Pivot rows of block q of the current matrix, minus the selector, into
// Vt[u][c] = M(8q + u, c) - [c == 8q + u] for every column c < NP.  Rows of
// the pivot tile row come from the tiles left of the diagonal; entries right
// of it from the column of tiles below (M is symmetric).
template <int NT, int WV>
__device__ __forceinline__ void publish_rows(const dbl4 (&acc)[SweepTiles<NT>::TPW], int q, double* Vt) {
    constexpr int NP = SweepTiles<NT>::NP;
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    const int tq = q >> 1, hq = q & 1;
#pragma unroll
    for (int k = 0; k < SweepTiles<NT>::TPW; ++k) {
        if (!slot_ok<NT>(WV, k)) continue;
        const int rt = slot_rt<NT>(WV, k), ct = slot_ct<NT>(WV, k);
        if (rt == tq) {
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) {
                const double v = hq ? acc[k][2 + jj] : acc[k][jj];
                const int u = 4 * jj + lr, c = 16 * ct + lc;
                Vt[u * NP + c] = v - (c == 8 * q + u ? 1.0 : 0.0);
            }
        } else if (ct == tq && rt > tq && (lc >> 3) == hq) {
            const int u = lc - 8 * hq;
#pragma unroll
            for (int j = 0; j < 4; ++j) Vt[u * NP + 16 * rt + 4 * j + lr] = acc[k][j];
        }
    }
}

// One block step on this wavefront's tiles: Z = V^T (V V~) on its two tile
// columns (rows 8..15 of each product are zero; D rows 0-3 and 4-7 are the
// B operands of the two K = 4 steps), then acc -= U~ Z and -2 on the swept
// diagonal.
template <int NT, int WV>
__device__ __forceinline__ void update_tiles(dbl4 (&acc)[SweepTiles<NT>::TPW], const double* __restrict__ V, const double* __restrict__ Vw,
                                             int q) {
    using T = SweepTiles<NT>;
    constexpr int NP = T::NP, TPW = T::TPW;
    constexpr int c1 = WV, c2 = 2 * kSweepWaves - 1 - WV;
    constexpr bool has2 = T::n2(WV) > 0;
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    double a1[2], a2[2], v1[2], v2[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int j = 4 * s + lr;
        a1[s] = (lc < 8 && j <= lc) ? Vw[tri8(lc) + j] : 0.0;   // V[lc][j]
        a2[s] = (lc < 8 && lc <= j) ? Vw[tri8(j) + lc] : 0.0;   // V[j][lc]
        v1[s] = V[j * NP + 16 * c1 + lc];
        v2[s] = has2 ? V[j * NP + 16 * c2 + lc] : 0.0;
    }
    double ua[TPW][2];
#pragma unroll
    for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int s = 0; s < 2; ++s)
            ua[k][s] = slot_ok<NT>(WV, k) ? -V[(4 * s + lr) * NP + 16 * slot_rt<NT>(WV, k) + lc] : 0.0;
    const dbl4 zero = {0.0, 0.0, 0.0, 0.0};
    dbl4 t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[0], v1[0], zero, 0, 0, 0);
    dbl4 t2 = zero;
    if constexpr (has2) t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[0], v2[0], zero, 0, 0, 0);
    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[1], v1[1], t1, 0, 0, 0);
    if constexpr (has2) t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[1], v2[1], t2, 0, 0, 0);
    dbl4 z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[0], t1[0], zero, 0, 0, 0);
    dbl4 z2 = zero;
    if constexpr (has2) z2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[0], t2[0], zero, 0, 0, 0);
    z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[1], t1[1], z1, 0, 0, 0);
    if constexpr (has2) z2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[1], t2[1], z2, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int k = 0; k < TPW; ++k)
            if (slot_ok<NT>(WV, k))
                acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[k][s], slot_first<NT>(WV, k) ? z1[s] : z2[s], acc[k],
                                                              0, 0, 0);
    const int tq = q >> 1, hq = q & 1;
    const bool lane_diag = (lc >> 3) == hq && lr == (lc & 3);
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        if (slot_ok<NT>(WV, k) && slot_rt<NT>(WV, k) == slot_ct<NT>(WV, k) && tq == slot_rt<NT>(WV, k)) {
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[k][j] -= (lane_diag && j == (lc >> 2)) ? 2.0 : 0.0;
        }
    }
}

template <int NT, int WV>
__device__ __forceinline__ void fill_tiles(dbl4 (&acc)[SweepTiles<NT>::TPW], const double* __restrict__ gram, int RR,
                                           double eta) {
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
#pragma unroll
    for (int k = 0; k < SweepTiles<NT>::TPW; ++k) {   // every load issued before any use
        const int rt = slot_rt<NT>(WV, k), ct = slot_ct<NT>(WV, k);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 16 * rt + 4 * j + lr, c = 16 * ct + lc;
            const bool in = slot_ok<NT>(WV, k) && r < RR && c < RR;
            const double g = in ? gram[(int64_t)r * RR + c] : 0.0;
            acc[k][j] = g + (r == c ? (r < RR ? eta : 1.0) : 0.0);
        }
    }
}

template <int NT, int WV>
__device__ __forceinline__ void store_tiles(const dbl4 (&acc)[SweepTiles<NT>::TPW], double* __restrict__ hm, int RR) {
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
#pragma unroll
    for (int k = 0; k < SweepTiles<NT>::TPW; ++k) {
        if (!slot_ok<NT>(WV, k)) continue;
        const int rt = slot_rt<NT>(WV, k), ct = slot_ct<NT>(WV, k);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 16 * rt + 4 * j + lr, c = 16 * ct + lc;
            if (r < RR && c < RR) {
                hm[(int64_t)r * RR + c] = acc[k][j];
                if (rt != ct) hm[(int64_t)c * RR + r] = acc[k][j];
            }
        }
    }
}

#define TRK_BY_WAVE(CALL)                       \
    switch (w) {                                \
        case 0: CALL(0); break;                 \
        case 1: CALL(1); break;                 \
        case 2: CALL(2); break;                 \
        default: CALL(3); break;                \
    }

// -(gram + eta I)^{-1} into hm (RR x RR, row-major, both triangles), with
// the fallback ladder; flag: 0 ok, 1 damped, 2 failed.  256 threads.
template <int NT>
__global__ __launch_bounds__(256) void k_sweep(tr_desc d, ModeSrc ms, const double* __restrict__ gram,
                                               double damping, double* __restrict__ hm, int* __restrict__ flag,
                                               int32_t* status) {
    using T = SweepTiles<NT>;
    constexpr int NP = T::NP, TPW = T::TPW;
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    const int npiv = (RR + 7) >> 3;
    __shared__ __align__(16) double Vt[2][8 * NP];
    __shared__ __align__(16) double Vws[kSweepWaves][40];
    __shared__ double red[kSweepWaves];
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    double* Vw = Vws[w];

    dbl4 acc[TPW];
    int ok_at = -1;
    double base = 0.0;   // tr(h + damping I) / RR, needed only once a factorisation has failed
    for (int attempt = 0; attempt < 8; ++attempt) {
        if (attempt == 1) {
            double tr = 0.0;
            for (int c = tid; c < RR; c += 256) tr += gram[(int64_t)c * RR + c];
            base = (block_sum(tr, red) + damping * RR) / RR;
        }
        const double eta = attempt == 0 ? damping : damping + pow(10.0, (double)(attempt - 1 - 10)) * base;
#define TRK_FILL(WV) fill_tiles<NT, WV>(acc, gram, RR, eta)
        TRK_BY_WAVE(TRK_FILL)
#undef TRK_FILL
        __syncthreads();   // the previous attempt's readers are done with Vt
#define TRK_PUB0(WV) publish_rows<NT, WV>(acc, 0, Vt[0])
        TRK_BY_WAVE(TRK_PUB0)
#undef TRK_PUB0
        bool good = true;
        for (int q = 0; q < npiv; ++q) {
            __syncthreads();
            const double* V = Vt[q & 1];
            good = pivot_chol_inv(V, NP, q, Vw);
            if (!good) break;   // the same in every wavefront: same data, same code
            // lane 0's stores of V reach LDS before any lane reads them (the
            // LDS instructions of one wavefront complete in order)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#define TRK_UPD(WV)                                                              \
    update_tiles<NT, WV>(acc, V, Vw, q);                                         \
    if (q + 1 < npiv) publish_rows<NT, WV>(acc, q + 1, Vt[(q + 1) & 1])
            TRK_BY_WAVE(TRK_UPD)
#undef TRK_UPD
        }
        if (good) {
            ok_at = attempt;
            break;
        }
    }
    if (ok_at >= 0) {
#define TRK_STORE(WV) store_tiles<NT, WV>(acc, hm, RR)
        TRK_BY_WAVE(TRK_STORE)
#undef TRK_STORE
    }
    if (tid == 0) {
        const int fl = ok_at < 0 ? 2 : (ok_at > 0 ? 1 : 0);
        *flag = fl;
        if (fl == 1) set_status(status, TR_DEV_DAMPED);
        if (fl == 2) set_status(status, TR_DEV_NOT_SPD);
    }
}

#undef TRK_BY_WAVE

constexpr int kApplyRows = 16;

// p = g (-M^{-1}) for 16 rows of g per block, then the rule.  Product on
// FP64 matrix cores: wavefront w owns the 16 x 16 output tiles of columns
// 16n.., n = w and w + 4; every operand (the block's rows of g, the
// columns of -M^{-1} it needs, the core and accumulator entries it updates)
// is loaded straight from global memory with all loads in flight, K padded
// with zeros to 128.  With lp.part set, block 0 also writes the loss.  With
// ``step`` set, the block that finishes last advances the step counter
// (after every block has read it).
template <typename TC>
__global__ __launch_bounds__(256) void k_scaled_apply(tr_desc d, ModeSrc ms, const TC* __restrict__ g,
                                                      LossParts lp, double* __restrict__ loss,
                                                      const double* __restrict__ hm, const int* __restrict__ flag,
                                                      MutPtrs cores, MutPtrs accum, tr_step rule, int32_t* status,
                                                      StepBump step) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    const int tid = threadIdx.x, l = tid & 63, lr = l & 15, lk = l >> 4, w = tid >> 6;
    __shared__ double red[4];
    if (blockIdx.x == 0 && lp.part) {
        const double s = loss_parts_sum(lp, In, red);
        if (tid == 0) *loss = s;
    }
    constexpr int KS = 32;                          // K steps of 4: RR <= 128
    const int r0 = blockIdx.x * kApplyRows;
    const int NTc = (RR + 15) >> 4;
    const int fl = *flag;
    TC* G = static_cast<TC*>(cores.p[n]);
    TC* A = static_cast<TC*>(accum.p[n]);
    // every operand in flight together: one wait on memory per block
    double a[KS], b[2][KS];                          // g[r0 + lr][4ks + lk], (-M^{-1})[4ks + lk][c]
    {
        const int row = r0 + lr;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k = 4 * ks + lk;
            a[ks] = (row < In && k < RR) ? (double)g[(int64_t)row * RR + k] : 0.0;
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = 16 * (w + 4 * u) + lr;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k = 4 * ks + lk;
            b[u][ks] = (k < RR && c < RR) ? hm[(int64_t)k * RR + c] : 0.0;
        }
    }
    double gold[2][4], aold[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * j + lk, c = 16 * (w + 4 * u) + lr;
            const bool in = r < In && c < RR;
            gold[u][j] = in ? (double)G[(int64_t)r * RR + c] : 0.0;
            aold[u][j] = (in && rule.kind == 1) ? (double)A[(int64_t)r * RR + c] : 0.0;
        }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int nt = w + 4 * u;
        const int c = 16 * nt + lr;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[u][ks], acc, 0, 0, 0);
        if (fl != 2 && nt < NTc) {   // fl == 2: not positive definite even with damping, core unchanged
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + 4 * j + lk;
                if (r < In && c < RR)
                    apply_rule_loaded<TC>(G, A, (int64_t)r * RR + c, gold[u][j], aold[u][j], acc[j], rule, t, status);
            }
        }
    }
    bump_if_last(step);
}

bool sweep_supported(const tr_desc& d) { return shape_of(d).maxRR <= 128; }

hipError_t launch_sweep_inverse(const tr_desc& d, ModeSrc ms, const double* gram, double damping, const UpdWs& L,
                                void* ws, int32_t* status, hipStream_t st) {
    const Shape sh = shape_of(d);
    if (sh.maxRR > 128) return hipErrorInvalidValue;
    char* w = static_cast<char*>(ws);
    double* hm = reinterpret_cast<double*>(w + L.L_off);
    int* flag = reinterpret_cast<int*>(w + L.flag_off);
    const int nt = (sh.maxRR + 15) / 16;
#define TRK_SWEEP(NTV) \
    hipLaunchKernelGGL(k_sweep<NTV>, dim3(1), dim3(256), 0, st, d, ms, gram, damping, hm, flag, status)
    switch (nt) {
        case 1: TRK_SWEEP(1); break;
        case 2: TRK_SWEEP(2); break;
        case 3: TRK_SWEEP(3); break;
        case 4: TRK_SWEEP(4); break;
        case 5: TRK_SWEEP(5); break;
        case 6: TRK_SWEEP(6); break;
        case 7: TRK_SWEEP(7); break;
        default: TRK_SWEEP(8); break;
    }
#undef TRK_SWEEP
    return hipGetLastError();
}

hipError_t launch_sweep_apply(const tr_desc& d, ModeSrc ms, const void* g, LossParts lp, double* loss, MutPtrs cores,
                              MutPtrs accum, tr_step rule, int32_t* status, void* ws, const UpdWs& L, StepBump step,
                              hipStream_t st) {
    const Shape sh = shape_of(d);
    if (sh.maxRR > 128) return hipErrorInvalidValue;
    char* w = static_cast<char*>(ws);
    const double* hm = reinterpret_cast<const double*>(w + L.L_off);
    const int* flag = reinterpret_cast<const int*>(w + L.flag_off);
    const dim3 grid((sh.maxI + kApplyRows - 1) / kApplyRows);
    if (d.core_dtype == TR_F64)
        hipLaunchKernelGGL(k_scaled_apply<double>, grid, dim3(256), 0, st, d, ms, static_cast<const double*>(g), lp,
                           loss, hm, flag, cores, accum, rule, status, step);
    else
        hipLaunchKernelGGL(k_scaled_apply<float>, grid, dim3(256), 0, st, d, ms, static_cast<const float*>(g), lp,
                           loss, hm, flag, cores, accum, rule, status, step);
    return hipGetLastError();
}

hipError_t launch_sweep_update(const tr_desc& d, ModeSrc ms, const double* gram, double damping, const void* g,
                               double* loss, MutPtrs cores, MutPtrs accum, tr_step rule, int32_t* status, void* ws,
                               const UpdWs& L, StepBump step, hipStream_t st) {
    hipError_t e = launch_sweep_inverse(d, ms, gram, damping, L, ws, status, st);
    if (e != hipSuccess) return e;
    return launch_sweep_apply(d, ms, g, LossParts{}, loss, cores, accum, rule, status, ws, L, step, st);
}

}  // namespace trk
