// a5/a6 on the matrix cores: fused fiber gather + prediction + residual +
// gradient contraction, FP32 in and out, v_mfma_f32_16x16x4_f32.
//
// Block = 4 wavefronts = 64 rows of G_{n(2)} (16 per wavefront) x a group
// of 64-sample chunks.  Per chunk:
//   GEMM1  P = G S^T      (64 x 64, K = R_n R_{n+1})  A = G rows (registers,
//                                                     loaded once), B = S (LDS)
//   E      = X_F - P      fibers read straight from HBM, each lane 4 rows of
//                         one fiber; scaled by -1/(m J_n p_f); E -> LDS
//   GEMM2  g += E S       (64 x RR, K = 64 samples)   A = E (LDS), B = S (LDS)
// The g tile stays in accumulators across the group's chunks and is written
// once as a partial sum; partials are added in a fixed order afterwards.
//
// Operand layouts of v_mfma_f32_16x16x4_f32 (one wavefront, lane l):
//   A: A[l % 16][l / 16]   B: B[l / 16][l % 16]   D: D[4 (l / 16) + j][l % 16], j < 4.
#include "wide.hpp"

namespace trk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfTI = 64;

// Row pitch of the staged S chunk: >= RRc and = 20 (mod 64) so that the
// 16 x 4 lane patterns of both GEMMs fall in distinct LDS banks.
__host__ __device__ constexpr int mf_pitch(int RRc) { return RRc + ((20 - RRc % 64) + 64) % 64; }

template <typename TX, int CT, int TF>
__global__ __launch_bounds__(256) void k_grad_mfma_f32(tr_desc d, ModeSrc ms, Ptrs cores, XSrc xsrc,
                                                       const int32_t* __restrict__ idx, const float* __restrict__ S,
                                                       const double* __restrict__ pF, int m, int groups,
                                                       int row_tiles_max, float* __restrict__ gpart,
                                                       double* __restrict__ lpart, int maxIRR, int rr_fixed) {
    int rtile, sgrp;
    if (!xcd_tile_group(row_tiles_max, groups, rtile, sgrp)) return;
    const int N = d.N;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    constexpr int SB = (16 * CT + 63) / 64;   // 64-column strips of a staged row
    constexpr int EP = TF + 4;   // row pitch of the staged E tile
    const int nchunks = (m + TF - 1) / TF;
    const int cpg = (nchunks + groups - 1) / groups;
    const int cbeg = sgrp * cpg, cend = min(nchunks, cbeg + cpg);
    // The next chunk's operands are held in registers until its turn: S rows
    // (TF / 4 per wavefront), the sample's indices and probability (every
    // thread loads those of sample tid % TF; the first TF use them).  Clamped
    // indices, no load behind a branch.
    float v[TF / 4][SB];
    int ik[kMaxOrder];
    double pf = 1.0;
    auto load_chunk = [&](int ch, int RRl) {
        const int f0 = ch * TF;
#pragma unroll
        for (int a = 0; a < TF / 4; ++a) {
            const int f = f0 + w + 4 * a;
            const float* src = S + (int64_t)(f < m ? f : m - 1) * RRl;
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int c = l + 64 * b;
                v[a][b] = src[c < RRl ? c : RRl - 1];
            }
        }
        const int fi = f0 + (tid & (TF - 1));
        const int64_t fc = fi < m ? fi : m - 1;
#pragma unroll
        for (int k = 0; k < kMaxOrder; ++k) ik[k] = idx[fc * N + (k < N ? k : N - 1)];
        pf = pF[fc];
    };
    // With one R_n R_{n+1} for every mode the first chunk's loads go out
    // before the step's mode has arrived.
    if (rr_fixed > 0 && cbeg < cend) load_chunk(cbeg, rr_fixed);
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, N)];
    // Tiles are fixed at compile time (CT column tiles of 16, KQ = 4 CT steps
    // of K = 4) and every matrix instruction runs unconditionally on
    // zero-padded operands: a run-time guard around an MFMA makes the compiler
    // move the accumulators between registers around every instruction.
    constexpr int KQ = 4 * CT, RRT = 16 * CT;
    constexpr int RRs = mf_pitch(RRT);
    const int i0 = rtile * kMfTI;
    if (i0 >= In) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* sS = reinterpret_cast<float*>(smem_raw);             // [TF][RRs]
    float* sE = sS + TF * RRs;                                  // [TI][EP]
    float* sW = sE + kMfTI * EP;                                // [TF]
    double* sL = reinterpret_cast<double*>(sW + TF);            // [TF]
    int64_t* sB = reinterpret_cast<int64_t*>(sL + TF);          // [TF]

    // A operand of GEMM1: this lane's G row, K in steps of 4.
    const float* Gn = static_cast<const float*>(cores.p[n]);
    // Loads at clamped indices, masked afterwards (no load behind a branch).
    const int grow = i0 + 16 * w + lr, growc = grow < In ? grow : In - 1;
    float ag[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        const int k = 4 * q + lk, kc = k < RR ? k : RR - 1;
        ag[q] = Gn[(int64_t)growc * RR + kc];
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q) ag[q] *= (grow < In && 4 * q + lk < RR) ? 1.f : 0.f;
    const bool rep = xsrc.rep[n] != nullptr;
    const TX* X = static_cast<const TX*>(rep ? xsrc.rep[n] : xsrc.X);
    int64_t xs[kMaxOrder];
    if (rep) {
        int64_t s = d.I[n];
        xs[n] = 1;
        int k = n;
        for (int q = 1; q < N; ++q) {
            k = ring_next(k, N);
            xs[k] = s;
            s *= d.I[k];
        }
    } else {
        for (int k = 0; k < N; ++k) xs[k] = d.x_stride[k];
    }
    const int64_t xsn = xs[n];

    f32x4 acc2[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc2[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    double lsum = 0.0;
    const double wbase = 1.0 / ((double)m * (double)J_of(d, n));
    const int erow = 16 * w + 4 * lk;   // first of this lane's 4 D rows (block-local)

    if (rr_fixed <= 0 && cbeg < cend) load_chunk(cbeg, RR);
    for (int ch = cbeg; ch < cend; ++ch) {
        const int f0 = ch * TF;
        __syncthreads();
        // the staged chunk into LDS
#pragma unroll
        for (int a = 0; a < TF / 4; ++a)
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int c = l + 64 * b;
                const bool ok = f0 + w + 4 * a < m && c < RR;
                if (c < RRT) sS[(w + 4 * a) * RRs + c] = ok ? v[a][b] : 0.f;
            }
        if (tid < TF) {
            const int f = f0 + tid;
            bool ok = f < m;
            int64_t off = 0;
            int ikm[kMaxOrder];
#pragma unroll
            for (int k = 0; k < kMaxOrder; ++k) ikm[k] = (ok && k < N) ? ik[k] : 0;
#pragma unroll
            for (int k = 0; k < kMaxOrder; ++k) {
                if (k >= N || k == n) continue;
                if (ikm[k] < 0 || ikm[k] >= d.I[k]) ok = false;
                off += (int64_t)ikm[k] * xs[k];
            }
            sB[tid] = ok ? off : 0;
            sW[tid] = ok ? (float)(wbase / pf) : 0.f;
            sL[tid] = ok ? 1.0 / (2.0 * (double)m * pf) : 0.0;
        }
        __syncthreads();
        // Fiber entries this lane needs, loaded before GEMM1 so that the HBM
        // latency overlaps the matrix-core work (clamped, branch-free).
        constexpr int NU = TF / 16;   // 16-sample tiles of the chunk
        float xv[NU][4];
        if (xsn == 1 && (In & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & (4 * sizeof(TX) - 1)) == 0) {
            // contiguous fibers and whole 4-row groups: one 4-wide load per
            // sample (aligned: every fiber offset is a multiple of I_n)
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int fl = 16 * u + lr;
                const bool ok4 = sW[fl] != 0.f && i0 + erow < In;
                load4(X + (ok4 ? sB[fl] + i0 + erow : 0), xv[u]);
            }
        } else {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int fl = 16 * u + lr;
                const bool okf = sW[fl] != 0.f;
                const int64_t base = sB[fl];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = i0 + erow + j;
                    const int64_t o = (okf && row < In) ? base + (int64_t)row * xsn : 0;
                    xv[u][j] = (float)to_f64(X[o]);
                }
            }
        }
        // the next chunk's operands, in flight during this chunk's products
        if (ch + 1 < cend) load_chunk(ch + 1, RR);

        // GEMM1: P[16w + 4lk + j][16t + lr]
        f32x4 p[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) p[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const float a = ag[q];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const float b = sS[(16 * u + lr) * RRs + 4 * q + lk];
                p[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, p[u], 0, 0, 0);
            }
        }
        // E = X_F - P, scaled; loss estimate
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int fl = 16 * u + lr;
            const float wf = sW[fl];
            const double lf = sL[fl];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool ok = (i0 + erow + j < In) && wf != 0.f;
                const float e = ok ? xv[u][j] - p[u][j] : 0.f;
                lsum += (double)e * (double)e * lf;
                sE[(erow + j) * EP + fl] = -e * wf;
            }
        }
        __syncthreads();
        // GEMM2: g[16w + 4lk + j][16ct + lr] += sum_f E[.][f] S[f][.]
#pragma unroll
        for (int q = 0; q < TF / 4; ++q) {
            const float a = sE[(16 * w + lr) * EP + 4 * q + lk];
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const float b = sS[(4 * q + lk) * RRs + 16 * c + lr];
                acc2[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc2[c], 0, 0, 0);
            }
        }
    }
    float* out = gpart + (int64_t)sgrp * maxIRR;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int col = 16 * c + lr;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = i0 + erow + j;
            if (row < In && col < RR) out[(int64_t)row * RR + col] = acc2[c][j];
        }
    }
    __shared__ double red[4];
    const double tot = block_sum(lsum, red);
    if (tid == 0) lpart[(int64_t)sgrp * row_tiles_max + rtile] = tot;
}

// ------------------------------------------------------------------------
// Wide-operand form, for R_n R_{n+1} a multiple of 4 in (32, 16 CT] (CT <= 8)
// with S and G_{n(2)} 16-byte aligned.  The kernel above is bound by the
// number of memory instructions, not by bytes or matrix-core time: one
// float per lane per load, LDS write and LDS read.  Here every one of them
// moves 16 bytes:
//   staging   LDS rows of S have the compile-time pitch SP = 4 Q words,
//             Q = 4 CT + 1 pieces of 16 bytes (Q odd: eight rows read
//             together by eight lanes start in distinct groups of four banks;
//             a run-time pitch would cost a register per operand address).
//             Piece k of staged row f is piece f RR/4 + k of the chunk's
//             rows in memory, so pieces past RR/4 continue into the next row
//             and the staged area is a flat copy: piece e at byte 16 e, moved
//             by direct memory-to-LDS loads (no registers, no LDS stores).
//   GEMM1     K order: lane group lk (= l / 16) owns k = 4 CT lk + q for its K
//             steps q < 4 CT, so four consecutive steps are one 16-byte read
//             of an S row and the A operand (the lane's G row) is CT 16-byte
//             loads; G is zero for k >= RR.
//   GEMM2     output column of tile c and lane column lr: CW lr + c, so the B
//             operands of one K step are CW consecutive floats of an S row;
//             K order: lane group lk owns samples TF/4 lk + s, so the A operand
//             (the residual, staged per wavefront as rows x samples) is read
//             16 bytes at a time as well.  Columns >= RR are computed and
//             dropped.
// The residual never leaves its wavefront (no barrier between the products).
// The products read up to 16 CT (GEMM1) and 16 CW (GEMM2) words from a row
// start; the words of a row past RR (the next row's entries, staged pieces
// past the last row, or the last piece of S where the addresses are
// clamped) meet a zero of G or feed a dropped column, and every one is a
// finite entry of S.  Rows past m hold such entries too; their residual is
// zero.
template <int CT>
struct WideCfg {
    static constexpr int TF = kWideTF;
    static constexpr int CW = CT <= 4 ? 4 : 8;        // GEMM2 column tiles
    static constexpr int Q = 4 * CT + 1;               // 16-byte pieces per staged row (odd)
    static constexpr int SP = 4 * Q;                   // staged row pitch in words
    static constexpr int TAIL = 16 * CW > SP ? 16 * CW - SP : 0;   // words read past the last row
    // staged pieces: TF rows and the tail, in whole wavefront instructions
    static constexpr int STAGE = (TF * Q + (TAIL + 3) / 4 + 63) / 64 * 64;
    static constexpr int EP = TF + 4;                  // residual row pitch (EP / 4 odd)
    static constexpr size_t shm() {
        return (size_t)STAGE * 16 + (size_t)(4 * 16 * EP + TF) * 4 + (size_t)TF * 16 + 64;
    }
};

template <typename TX, int CT>
__global__ __launch_bounds__(256) void k_grad_mfma_f32w(tr_desc d, ModeSrc ms, Ptrs cores, XSrc xsrc,
                                                        const int32_t* __restrict__ idx, const float* __restrict__ S,
                                                        const double* __restrict__ pF, int m, int groups,
                                                        int row_tiles_max, float* __restrict__ gpart,
                                                        double* __restrict__ lpart, int maxIRR, int rr_fixed,
                                                        WideModes tab) {
    using C = WideCfg<CT>;
    constexpr int TF = C::TF, CW = C::CW, EP = C::EP, SP = C::SP, NU = TF / 16, TQ = TF / 4;
    int rtile, sgrp;
    if (!xcd_tile_group(row_tiles_max, groups, rtile, sgrp)) return;
    const int N = d.N;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    // One chunk of TF samples per sample group (the launcher has as many
    // groups as chunks; a group past the last sample writes a zero partial).
    const int f0 = sgrp * TF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* sS = reinterpret_cast<float*>(smem_raw);                 // [STAGE pieces]
    float* sE = sS + 4 * C::STAGE;                                  // [4][16][EP]
    float* sW = sE + 4 * 16 * EP;                                   // [TF], lane order
    double* sL = reinterpret_cast<double*>(sW + TF);                // [TF], lane order
    int64_t* sB = reinterpret_cast<int64_t*>(sL + TF);              // [TF], lane order
    // The chunk's pieces of S (straight into LDS) and its samples' indices
    // and probabilities go out first: before the step's mode is known when
    // every mode has the same R_n R_{n+1}, and in one batch with the core
    // rows otherwise, so that the block waits for memory once.  Clamped
    // in-bounds addresses.
    const int wu = __builtin_amdgcn_readfirstlane(w);   // the wavefront index, in a scalar register
    WideSample smp;
    auto issue = [&](int RRl) {
        const int q0 = RRl >> 2;
        wide_stage<C::Q, C::STAGE>(S, sS, q0, f0 * q0, m * q0 - 1, wu, l);   // < 2^30 pieces
        smp = wide_sample_load(idx, pF, f0, m, N);
    };
    uint64_t t;
    int n = 0;
    if (rr_fixed <= 0) resolve_mode(ms, N, &t, &n);
    issue(rr_fixed > 0 ? rr_fixed : d.R[n] * d.R[ring_next(n, N)]);
    if (rr_fixed > 0) resolve_mode(ms, N, &t, &n);
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, N)];
    const WideMode& wm = tab.md[n];
    const int i0 = rtile * kMfTI;
    if (i0 >= In) {
        __builtin_amdgcn_s_waitcnt(0);   // no direct load outlives the block
        return;
    }
    float* sEw = sE + w * 16 * EP;

    // A operand of GEMM1: the lane's G row, K steps 4j..4j+3 in one piece
    // (masked once the pieces of S are in LDS).
    const float* Gn = static_cast<const float*>(cores.p[n]);
    const int grow = i0 + 16 * w + lr, growc = grow < In ? grow : In - 1;
    float4 ga[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        const int k0 = 4 * CT * lk + 4 * j;
        ga[j] = *reinterpret_cast<const float4*>(Gn + (int64_t)growc * RR + (k0 < RR ? k0 : 0));
    }
    const TX* X = static_cast<const TX*>(xsrc.rep[n] ? xsrc.rep[n] : xsrc.X);
    const int64_t xsn = xsrc.rep[n] ? 1 : d.x_stride[n];
    const bool fast_fiber = wm.fast != 0;
    const int erow = 16 * w + 4 * lk;   // first of this lane's 4 D rows (block-local)

    // each sample's fiber offset and weights, in lane order
    wide_sample_meta(smp, d, wm, n, f0, m, sB, sW, sL);
#pragma unroll
    for (int j = 0; j < CT; ++j) ga[j] = mask4(ga[j], grow < In && 4 * CT * lk + 4 * j < RR);
    __builtin_amdgcn_s_waitcnt(0);   // this wavefront's direct loads have landed
    __syncthreads();
    // fiber entries of this lane's 4 rows, in flight during GEMM1
    float wv[NU];
    int64_t bv[NU];
#pragma unroll
    for (int h = 0; h < NU / 4; ++h) {
        const float4 q = *reinterpret_cast<const float4*>(sW + 8 * lr + 4 * h);
        wv[4 * h] = q.x;
        wv[4 * h + 1] = q.y;
        wv[4 * h + 2] = q.z;
        wv[4 * h + 3] = q.w;
    }
#pragma unroll
    for (int h = 0; h < NU / 2; ++h) {
        const longlong2 q = *reinterpret_cast<const longlong2*>(sB + 8 * lr + 2 * h);
        bv[2 * h] = q.x;
        bv[2 * h + 1] = q.y;
    }
    float xv[NU][4];
    if (fast_fiber) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const bool ok4 = wv[u] != 0.f && i0 + erow < In;
            load4(X + (ok4 ? bv[u] + i0 + erow : 0), xv[u]);
        }
    } else {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = i0 + erow + j;
                const int64_t o = (wv[u] != 0.f && row < In) ? bv[u] + (int64_t)row * xsn : 0;
                xv[u][j] = (float)to_f64(X[o]);
            }
        }
    }
    // GEMM1: P[erow + j][16u + lr], K step q of group lk is k = 4 CT lk + q
    // (piece j of the K range outer, the 8 sample tiles inner: 32
    // independent products per 8 reads)
    // (piece j + 1's reads go out before piece j's products, in the order
    // the scheduling groups keep)
    __builtin_amdgcn_sched_barrier(0);
    f32x4 p[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) p[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    const float* srow = sS + lr * SP + 4 * CT * lk;
    float4 bc[NU], bn[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) bc[u] = *reinterpret_cast<const float4*>(srow + 16 * u * SP);
    __builtin_amdgcn_sched_group_barrier(0x100, NU, 0);
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        if (j + 1 < CT) {
#pragma unroll
            for (int u = 0; u < NU; ++u) bn[u] = *reinterpret_cast<const float4*>(srow + 16 * u * SP + 4 * (j + 1));
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) p[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[j].x, bc[u].x, p[u], 0, 0, 0);
#pragma unroll
        for (int u = 0; u < NU; ++u) p[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[j].y, bc[u].y, p[u], 0, 0, 0);
#pragma unroll
        for (int u = 0; u < NU; ++u) p[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[j].z, bc[u].z, p[u], 0, 0, 0);
#pragma unroll
        for (int u = 0; u < NU; ++u) p[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[j].w, bc[u].w, p[u], 0, 0, 0);
        if (j + 1 < CT) __builtin_amdgcn_sched_group_barrier(0x100, NU, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * NU, 0);
        if (j + 1 < CT) {
#pragma unroll
            for (int u = 0; u < NU; ++u) bc[u] = bn[u];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // E = X_F - P, scaled; loss estimate; E into the wavefront's rows
    double lsum = 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int fl = 16 * u + lr;
        const float wf = wv[u];
        const double lf = sL[8 * lr + u];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool ok = (i0 + erow + j < In) && wf != 0.f;
            const float e = ok ? xv[u][j] - p[u][j] : 0.f;
            lsum += (double)e * (double)e * lf;
            sEw[(4 * lk + j) * EP + fl] = -e * wf;
        }
    }
    // GEMM2: g[erow + j][col(c)] += sum_s E[.][TQ lk + s] S[TQ lk + s][col(c)]
    // for the lane's CW columns col(c) = 64 (c / 4) + 4 lr + c % 4: each
    // 16-byte read of S covers 64 consecutive columns across 16 lanes, so
    // no two lanes of a read share an LDS bank (columns CW lr + c put lanes
    // lr and lr + 4 in one bank when CW = 8)
    // (the residual rows are this wavefront's own: LDS operations of a
    // wavefront complete in order, so no barrier)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_sched_barrier(0);   // GEMM2's issue order below stays its own
    f32x4 acc2[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc2[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    // K step s + 1's operands are read before step s's products, and the
    // scheduling groups keep that order (left alone, the compiler reads
    // each step's operands right before they are used).
    const float* erw = sEw + lr * EP + TQ * lk;
    const float* scl = sS + (TQ * lk) * SP + 4 * lr;
    constexpr int RPS = CW / 4;   // 16-byte B reads per K step
    float4 acur = *reinterpret_cast<const float4*>(erw), anxt = acur;
    float4 bcur[RPS], bnxt[RPS];
#pragma unroll
    for (int h = 0; h < RPS; ++h) bcur[h] = *reinterpret_cast<const float4*>(scl + 64 * h);
    __builtin_amdgcn_sched_group_barrier(0x100, 1 + RPS, 0);
#pragma unroll
    for (int st = 0; st < TQ; ++st) {
        if (st + 1 < TQ) {
#pragma unroll
            for (int h = 0; h < RPS; ++h) bnxt[h] = *reinterpret_cast<const float4*>(scl + (st + 1) * SP + 64 * h);
            if ((st + 1) % 4 == 0) anxt = *reinterpret_cast<const float4*>(erw + (st + 1));
        }
        const float at = (st & 3) == 0 ? acur.x : (st & 3) == 1 ? acur.y : (st & 3) == 2 ? acur.z : acur.w;
#pragma unroll
        for (int h = 0; h < RPS; ++h) {
            acc2[4 * h] = __builtin_amdgcn_mfma_f32_16x16x4f32(at, bcur[h].x, acc2[4 * h], 0, 0, 0);
            acc2[4 * h + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(at, bcur[h].y, acc2[4 * h + 1], 0, 0, 0);
            acc2[4 * h + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(at, bcur[h].z, acc2[4 * h + 2], 0, 0, 0);
            acc2[4 * h + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(at, bcur[h].w, acc2[4 * h + 3], 0, 0, 0);
        }
        if (st + 1 < TQ && (st + 1) % 4 == 0) __builtin_amdgcn_sched_group_barrier(0x100, RPS + 1, 0);
        if (st + 1 < TQ && (st + 1) % 4 != 0) __builtin_amdgcn_sched_group_barrier(0x100, RPS, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, CW, 0);
#pragma unroll
        for (int h = 0; h < RPS; ++h) bcur[h] = bnxt[h];
        if ((st + 1) % 4 == 0) acur = anxt;
    }
    float* out = gpart + (int64_t)sgrp * maxIRR;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = i0 + erow + j;
#pragma unroll
        for (int h = 0; h < CW / 4; ++h) {
            const int col = 64 * h + 4 * lr;
            if (row < In && col < RR)
                *reinterpret_cast<float4*>(out + (int64_t)row * RR + col) =
                    make_float4(acc2[4 * h][j], acc2[4 * h + 1][j], acc2[4 * h + 2][j], acc2[4 * h + 3][j]);
        }
    }
    __shared__ double red[4];
    const double ws = wave_sum_dpp(lsum);
    if (l == 0) red[w] = ws;
    __syncthreads();
    if (tid == 0) lpart[(int64_t)sgrp * row_tiles_max + rtile] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <int CT, int TF>
static constexpr size_t grad_mfma_shm() {
    return (size_t)(TF * mf_pitch(16 * CT) + kMfTI * (TF + 4) + TF) * 4 + (size_t)TF * 16 + 64;
}

template <typename TX, int CT, int TF>
static hipError_t launch_ctf(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                             const double* pF, int m, dim3 grid, int groups, int row_tiles, float* gp, double* lp,
                             int maxIRR, hipStream_t st) {
    constexpr size_t shm = grad_mfma_shm<CT, TF>();
    if (!allow_lds(reinterpret_cast<const void*>(&k_grad_mfma_f32<TX, CT, TF>), shm)) return hipErrorInvalidValue;
    int rr_fixed = d.R[0] * d.R[1 % d.N];
    for (int k = 1; k < d.N; ++k)
        if (d.R[k] * d.R[(k + 1) % d.N] != rr_fixed) rr_fixed = 0;
    launch_timed(k_grad_mfma_f32<TX, CT, TF>, grid, dim3(256), shm, st, d, ms, cores, xs, idx, S, pF, m, groups,
                 row_tiles, gp, lp, maxIRR, rr_fixed);
    return hipGetLastError();
}

template <typename TX, int CT>
static hipError_t launch_wide(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                              const double* pF, int m, dim3 grid, int groups, int row_tiles, float* gp, double* lp,
                              int maxIRR, hipStream_t st) {
    constexpr size_t shm = WideCfg<CT>::shm();
    if (!allow_lds(reinterpret_cast<const void*>(&k_grad_mfma_f32w<TX, CT>), shm)) return hipErrorInvalidValue;
    const WideModes tab = wide_modes(d, xs, m, sizeof(TX));
    launch_timed(k_grad_mfma_f32w<TX, CT>, grid, dim3(256), shm, st, d, ms, cores, xs, idx, S, pF, m, groups,
                 row_tiles, gp, lp, maxIRR, wide_rr_fixed(d), tab);
    return hipGetLastError();
}

template <typename TX>
static hipError_t launch_wide_tx(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx,
                                 const float* S, const double* pF, int m, dim3 grid, int groups, int row_tiles,
                                 float* gp, double* lp, int maxIRR, int maxRR, hipStream_t st) {
    switch ((maxRR + 15) / 16) {
        case 3: return launch_wide<TX, 3>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 4: return launch_wide<TX, 4>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 5: return launch_wide<TX, 5>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 6: return launch_wide<TX, 6>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 7: return launch_wide<TX, 7>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 8: return launch_wide<TX, 8>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        default: return hipErrorInvalidValue;
    }
}

// Chunks of 128 samples (one pass per block over twice the samples, half
// the dependent staging rounds) for up to 8 column tiles; 64 otherwise.
template <typename TX, int CT>
static hipError_t launch_ct(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                            const double* pF, int m, dim3 grid, int groups, int row_tiles, float* gp, double* lp,
                            int maxIRR, int tf, hipStream_t st) {
    if constexpr (CT <= 8) {
        if (tf == 128)
            return launch_ctf<TX, CT, 128>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR,
                                           st);
    }
    return launch_ctf<TX, CT, 64>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
}

// Smallest compiled tile count covering ceil(maxRR / 16) column tiles.
template <typename TX>
static hipError_t launch_tx(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                            const double* pF, int m, dim3 grid, int groups, int row_tiles, float* gp, double* lp,
                            int maxIRR, int maxRR, int tf, hipStream_t st) {
    const int nct = (maxRR + 15) / 16;
#define TRK_CT(C)                                                                                              \
    if (nct <= C)                                                                                              \
    return launch_ct<TX, C>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, tf, st)
    TRK_CT(1);
    TRK_CT(2);
    TRK_CT(3);
    TRK_CT(4);
    TRK_CT(5);
    TRK_CT(6);
    TRK_CT(7);
    TRK_CT(8);
    TRK_CT(10);
    TRK_CT(12);
    TRK_CT(16);
#undef TRK_CT
    return hipErrorInvalidValue;
}

hipError_t launch_grad_mfma_f32(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx,
                                const float* S, const double* pF, int m, int groups, int row_tiles, float* gp,
                                double* lp, int tf, hipStream_t st) {
    const Shape sh = shape_of(d);
    const dim3 grid(xcd_grid(row_tiles, groups));
    const int maxIRR = sh.maxI * sh.maxRR;
    // (the 16-byte form takes one chunk of 128 samples per group whatever
    // chunk the layout chose: with 64-sample chunks m <= 64 groups, and a
    // group past the last sample writes a zero partial)
    if (wide_applies(d, cores, S, gp, m, groups, sh.maxRR, kWideTF)) {
        if (d.x_dtype == TR_F32)
            return launch_wide_tx<float>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR,
                                         sh.maxRR, st);
        if (d.x_dtype == TR_F16)
            return launch_wide_tx<__half>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR,
                                          sh.maxRR, st);
    }
    switch (d.x_dtype) {
        case TR_F32:
            return launch_tx<float>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR,
                                    sh.maxRR, tf, st);
        case TR_F16:
            return launch_tx<__half>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR,
                                     sh.maxRR, tf, st);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace trk
