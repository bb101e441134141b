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
#include "internal.hpp"

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
