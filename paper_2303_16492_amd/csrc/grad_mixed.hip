// a5/a6 in mixed precision: the fused fiber gather + prediction + residual +
// gradient contraction on 16-bit matrix cores (v_mfma_f32_16x16x32_bf16 or
// _f16) with FP32 accumulation.
//
// Precision policy (the paper fixes none):
//   GEMM1  P = G S^T  from hi/lo splits, G = Gh + Gl, S = Sh + Sl (each part
//          16-bit): P ~ Gh Sh + Gh Sl + Gl Sh, three products, about FP32
//          accuracy.  A single 16-bit product would leave an absolute error
//          ~2^-9 |X| in E = X_F - P that does not shrink as the fit improves.
//   E      rounded to 16 bits once (its error is relative to E itself).
//   GEMM2  g += E (Sh + Sl): two products, so the gradient and the Gram see
//          the same sampled rows to 16 mantissa bits (a scaled step built from
//          mismatched rows is off by that mismatch times the condition
//          number of the Gram).
//   Gram   FP64 (separate kernel), Cholesky FP64.
//
// Tiles as in the FP32 kernel: block = 4 wavefronts = 64 rows x groups of
// 64-sample chunks.  Operand layouts of v_mfma_f32_16x16x32_{bf16,f16}
// (lane l, 8 values per lane): A[l % 16][8 (l / 16) + i], B[8 (l / 16) + i][l % 16],
// D[4 (l / 16) + j][l % 16].  S is staged twice: row-major (B of GEMM1) and
// transposed (B of GEMM2), so every operand is one 16-byte LDS read.
#include "wide.hpp"

namespace trk {

typedef float f32x4m __attribute__((ext_vector_type(4)));

template <typename T16> struct Mf16;
template <> struct Mf16<__bf16> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    static __device__ inline f32x4m mma(v8 a, v8 b, f32x4m c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mf16<_Float16> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    static __device__ inline f32x4m mma(v8 a, v8 b, f32x4m c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

constexpr int kMxTI = 64, kMxTF = 64, kMxTP = kMxTF + 8;

template <int CT>
struct MixGeom {
    static constexpr int KS = (16 * CT + 31) / 32;   // K steps of 32 in GEMM1
    static constexpr int KP = 32 * KS + 8;           // row pitch of row-major S parts
    static constexpr int NC = 16 * CT;               // padded gradient columns
    static constexpr int SB = (32 * KS + 63) / 64;   // 64-column strips staged per row
    static constexpr size_t lds() {
        return (size_t)2 * (2 * kMxTF * KP + 2 * NC * kMxTP + kMxTI * kMxTP) + kMxTF * 4 + kMxTF * 16 + 64;
    }
};

template <typename T16, typename TX, int CT>
__global__ __launch_bounds__(256) void k_grad_mixed(tr_desc d, ModeSrc ms, Ptrs cores, XSrc xsrc,
                                                    const int32_t* __restrict__ idx, const float* __restrict__ S,
                                                    const double* __restrict__ pF, int m, int groups,
                                                    int row_tiles_max, float* __restrict__ gpart,
                                                    double* __restrict__ lpart, int maxIRR) {
    int rtile, sgrp;
    if (!xcd_tile_group(row_tiles_max, groups, rtile, sgrp)) return;
    typedef MixGeom<CT> Gm;
    typedef typename Mf16<T16>::v8 v8;
    constexpr int KS = Gm::KS, KP = Gm::KP, NC = Gm::NC, SB = Gm::SB;
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int N = d.N;
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, N)];
    const int i0 = rtile * kMxTI;
    if (i0 >= In) return;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    T16* sSh = reinterpret_cast<T16*>(smem_raw);   // [TF][KP]
    T16* sSl = sSh + kMxTF * KP;                   // [TF][KP]
    T16* sTh = sSl + kMxTF * KP;                   // [NC][TP]  (transposed)
    T16* sTl = sTh + NC * kMxTP;                   // [NC][TP]
    T16* sE = sTl + NC * kMxTP;                    // [TI][TP]
    float* sW = reinterpret_cast<float*>(sE + kMxTI * kMxTP);
    double* sL = reinterpret_cast<double*>(sW + kMxTF);
    int64_t* sB = reinterpret_cast<int64_t*>(sL + kMxTF);

    // A operand of GEMM1: this lane's G row split hi/lo, 8 values per K step.
    const float* Gn = static_cast<const float*>(cores.p[n]);
    // (loads at clamped indices, masked afterwards: none behind a branch)
    const int grow = i0 + 16 * w + lr, growc = grow < In ? grow : In - 1;
    float gv[KS][8];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 32 * s + 8 * lk + i;
            gv[s][i] = Gn[(int64_t)growc * RR + (k < RR ? k : RR - 1)];
        }
    v8 ah[KS], al[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 32 * s + 8 * lk + i;
            const float g = (grow < In && k < RR) ? gv[s][i] : 0.f;
            const T16 h = (T16)g;
            ah[s][i] = h;
            al[s][i] = (T16)(g - (float)h);
        }
    }
    const bool rep = xsrc.rep[n] != nullptr;
    const TX* X = static_cast<const TX*>(rep ? xsrc.rep[n] : xsrc.X);
    int64_t xs[kMaxOrder];
    if (rep) {
        int64_t sz = d.I[n];
        xs[n] = 1;
        int k = n;
        for (int q = 1; q < N; ++q) {
            k = ring_next(k, N);
            xs[k] = sz;
            sz *= d.I[k];
        }
    } else {
        for (int k = 0; k < N; ++k) xs[k] = d.x_stride[k];
    }
    const int64_t xsn = xs[n];

    f32x4m acc2[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc2[c] = f32x4m{0.f, 0.f, 0.f, 0.f};
    double lsum = 0.0;
    const double wbase = 1.0 / ((double)m * (double)J_of(d, n));
    const int nchunks = (m + kMxTF - 1) / kMxTF;
    const int cpg = (nchunks + groups - 1) / groups;
    const int cbeg = sgrp * cpg, cend = min(nchunks, cbeg + cpg);
    const int erow = 16 * w + 4 * lk;

    for (int ch = cbeg; ch < cend; ++ch) {
        const int f0 = ch * kMxTF;
        __syncthreads();
        {   // stage S split hi/lo, row-major and transposed; loads first
            float v[16][SB];
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                const int f = w + 4 * a;
                const float* src = S + (int64_t)(f0 + f < m ? f0 + f : m - 1) * RR;
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const int c = l + 64 * b;
                    v[a][b] = src[c < RR ? c : RR - 1];
                }
            }
#pragma unroll
            for (int a = 0; a < 16; ++a)
#pragma unroll
                for (int b = 0; b < SB; ++b)
                    if (!(f0 + w + 4 * a < m && l + 64 * b < RR)) v[a][b] = 0.f;
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                const int f = w + 4 * a;
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const int c = l + 64 * b;
                    const T16 h = (T16)v[a][b];
                    const T16 lo = (T16)(v[a][b] - (float)h);
                    if (c < 32 * KS) {
                        sSh[f * KP + c] = h;
                        sSl[f * KP + c] = lo;
                    }
                    if (c < NC) {
                        sTh[c * kMxTP + f] = h;
                        sTl[c * kMxTP + f] = lo;
                    }
                }
            }
        }
        if (tid < kMxTF) {
            const int f = f0 + tid;
            bool ok = f < m;
            int64_t off = 0;
            int ik[kMaxOrder];
            const int64_t fc = ok ? f : m - 1;
#pragma unroll
            for (int k = 0; k < kMaxOrder; ++k) ik[k] = idx[fc * N + (k < N ? k : N - 1)];
            const double pf = pF[fc];
#pragma unroll
            for (int k = 0; k < kMaxOrder; ++k) ik[k] = (ok && k < N) ? ik[k] : 0;
#pragma unroll
            for (int k = 0; k < kMaxOrder; ++k) {
                if (k >= N || k == n) continue;
                if (ik[k] < 0 || ik[k] >= d.I[k]) ok = false;
                off += (int64_t)ik[k] * xs[k];
            }
            sB[tid] = ok ? off : 0;
            sW[tid] = ok ? (float)(wbase / pf) : 0.f;
            sL[tid] = ok ? 1.0 / (2.0 * (double)m * pf) : 0.0;
        }
        __syncthreads();
        float xv[4][4];
        if (xsn == 1 && (In & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & (4 * sizeof(TX) - 1)) == 0) {
            // contiguous fibers and whole 4-row groups: one 4-wide load per
            // sample (aligned: every fiber offset is a multiple of I_n)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int fl = 16 * u + lr;
                const bool ok4 = sW[fl] != 0.f && i0 + erow < In;
                load4(X + (ok4 ? sB[fl] + i0 + erow : 0), xv[u]);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
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
        // GEMM1 (three products)
        f32x4m p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = f32x4m{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int off = (16 * u + lr) * KP + 32 * s + 8 * lk;
                const v8 bh = *reinterpret_cast<const v8*>(sSh + off);
                const v8 bl = *reinterpret_cast<const v8*>(sSl + off);
                p[u] = Mf16<T16>::mma(ah[s], bh, p[u]);
                p[u] = Mf16<T16>::mma(ah[s], bl, p[u]);
                p[u] = Mf16<T16>::mma(al[s], bh, p[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int fl = 16 * u + lr;
            const float wf = sW[fl];
            const double lf = sL[fl];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool ok = (i0 + erow + j < In) && wf != 0.f;
                const float e = ok ? xv[u][j] - p[u][j] : 0.f;
                lsum += (double)e * (double)e * lf;
                sE[(erow + j) * kMxTP + fl] = (T16)(-e * wf);
            }
        }
        __syncthreads();
        // GEMM2 (two products), K = 64 samples in two steps of 32
#pragma unroll
        for (int s = 0; s < kMxTF / 32; ++s) {
            const v8 a = *reinterpret_cast<const v8*>(sE + (16 * w + lr) * kMxTP + 32 * s + 8 * lk);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int off = (16 * c + lr) * kMxTP + 32 * s + 8 * lk;
                const v8 bh = *reinterpret_cast<const v8*>(sTh + off);
                const v8 bl = *reinterpret_cast<const v8*>(sTl + off);
                acc2[c] = Mf16<T16>::mma(a, bh, acc2[c]);
                acc2[c] = Mf16<T16>::mma(a, bl, acc2[c]);
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
// 16-byte-operand form (same conditions as the FP32 one: R_n R_{n+1} a
// multiple of 4 in (32, 16 CT], one chunk of 128 samples per sample group).
// The kernel above spends its time staging S as four 16-bit copies with one
// 2-byte LDS store per value and copy; here:
//   staging   the chunk's rows of S go straight into LDS as FP32 (direct
//             loads, a flat copy into rows of Q = 4 CT + 1 pieces).
//   split     S is split into 16-bit hi/lo once per block, in one pass: each
//             thread owns an 8 x 8 block of the staged chunk (8 samples x 8
//             entries), reads it with sixteen 16-byte reads, and writes it
//             back in place as rows of [8 hi][8 lo] (GEMM1's B operand) and
//             as 16-byte runs of 8 samples of S^T, hi and lo (GEMM2's B
//             operand needs 8 consecutive samples of one column per lane).
//             No other thread reads or writes the block's bytes.  Staged
//             rows have Q = 8 KS + 1 pieces so that the split K range fits.
//   GEMM1     three 16-bit products per K step of 32, both operands split
//             once (B: one 16-byte LDS read each for hi and lo).
//   GEMM2     two products over CW column tiles, column CW lr + c in tile c
//             (S^T row 16 c + lr holds column CW lr + c), so a lane's
//             results for one row are CW adjacent columns (16-byte stores);
//             the residual is rounded to 16 bits once and stays in its
//             wavefront's rows.
// Reads past R_n R_{n+1} (GEMM1's K up to 32 KS, S^T columns up to 16 CT)
// land on finite staged entries of the same row, which meet a zero of G
// or feed a dropped column.
template <int CT>
struct MixWideCfg {
    static constexpr int TF = kWideTF;
    static constexpr int KS = (16 * CT + 31) / 32;      // GEMM1 K steps of 32
    static constexpr int CW = CT <= 4 ? 4 : 8;          // GEMM2 column tiles
    static constexpr int NC = 16 * CW;                  // gradient columns (padded), S^T rows
    static constexpr int KW = 32 * KS > NC ? 32 * KS : NC;   // staged entries a row's split covers
    static constexpr int Q = KW / 4 + 1;                // 16-byte pieces per staged row (odd)
    static constexpr int SP = 4 * Q;                    // staged row pitch in words
    static constexpr int STAGE = (TF * Q + 63) / 64 * 64;
    static constexpr int TP = TF + 8;                   // row pitch (16-bit entries) of S^T parts and E
    static constexpr size_t lds() {
        return (size_t)STAGE * 16 + (size_t)2 * NC * TP * 2 + (size_t)kMxTI * TP * 2 + (size_t)TF * 4 +
               (size_t)TF * 16 + 64;
    }
};

// hi = 16-bit rounding of x, lo = 16-bit rounding of x - hi, two entries
// per conversion.
template <typename T16>
__device__ __forceinline__ void split8(const float (&x)[8], typename Mf16<T16>::v8& hi, typename Mf16<T16>::v8& lo) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef T16 h2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        const h2 h = __builtin_convertvector((f2){x[q], x[q + 1]}, h2);
        const h2 r = __builtin_convertvector((f2){x[q] - (float)h[0], x[q + 1] - (float)h[1]}, h2);
        hi[q] = h[0];
        hi[q + 1] = h[1];
        lo[q] = r[0];
        lo[q + 1] = r[1];
    }
}

template <typename T16, typename TX, int CT>
__global__ __launch_bounds__(256) void k_grad_mixed_w(tr_desc d, ModeSrc ms, Ptrs cores, XSrc xsrc,
                                                      const int32_t* __restrict__ idx, const float* __restrict__ S,
                                                      const double* __restrict__ pF, int m, int groups,
                                                      int row_tiles_max, float* __restrict__ gpart,
                                                      double* __restrict__ lpart, int maxIRR, int rr_fixed,
                                                      WideModes tab) {
    using C = MixWideCfg<CT>;
    typedef typename Mf16<T16>::v8 v8;
    constexpr int TF = C::TF, KS = C::KS, NC = C::NC, CW = C::CW, SP = C::SP, TP = C::TP, NU = TF / 16;
    int rtile, sgrp;
    if (!xcd_tile_group(row_tiles_max, groups, rtile, sgrp)) return;
    const int N = d.N;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int f0 = sgrp * TF;   // the group's chunk
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* sS = reinterpret_cast<float*>(smem_raw);                  // [STAGE pieces], FP32
    T16* sTh = reinterpret_cast<T16*>(sS + 4 * C::STAGE);            // [NC][TP]
    T16* sTl = sTh + NC * TP;                                        // [NC][TP]
    T16* sE = sTl + NC * TP;                                         // [64][TP]
    float* sW = reinterpret_cast<float*>(sE + kMxTI * TP);           // [TF], lane order
    double* sL = reinterpret_cast<double*>(sW + TF);                 // [TF], lane order
    int64_t* sB = reinterpret_cast<int64_t*>(sL + TF);               // [TF], lane order
    const int wu = __builtin_amdgcn_readfirstlane(w);
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
    const int i0 = rtile * kMxTI;
    if (i0 >= In) {
        __builtin_amdgcn_s_waitcnt(0);   // no direct load outlives the block
        return;
    }
    // A operand of GEMM1: the lane's G row, entries 32 s + 8 lk + i (two
    // 16-byte loads per K step), split hi/lo once the pieces of S are in.
    const float* Gn = static_cast<const float*>(cores.p[n]);
    const int grow = i0 + 16 * w + lr, growc = grow < In ? grow : In - 1;
    float4 gq[KS][2];
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k0 = 32 * s2 + 8 * lk + 4 * h;
            gq[s2][h] = *reinterpret_cast<const float4*>(Gn + (int64_t)growc * RR + (k0 < RR ? k0 : 0));
        }
    const TX* X = static_cast<const TX*>(xsrc.rep[n] ? xsrc.rep[n] : xsrc.X);
    const int64_t xsn = xsrc.rep[n] ? 1 : d.x_stride[n];
    const bool fast_fiber = wm.fast != 0;
    const int erow = 16 * w + 4 * lk;
    wide_sample_meta(smp, d, wm, n, f0, m, sB, sW, sL);
    v8 ah[KS], al[KS];
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2) {
        const float4 g0 = mask4(gq[s2][0], grow < In && 32 * s2 + 8 * lk < RR);
        const float4 g1 = mask4(gq[s2][1], grow < In && 32 * s2 + 8 * lk + 4 < RR);
        const float gv[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
        split8<T16>(gv, ah[s2], al[s2]);
    }
    __builtin_amdgcn_s_waitcnt(0);   // this wavefront's direct loads have landed
    __syncthreads();
    // fiber entries of this lane's 4 rows, in flight from here on
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
    // the split: block (g, b) = samples 8 g .. 8 g + 7, entries 8 b .. 8 b + 7
    constexpr int NBLK = (TF / 8) * (C::KW / 8);
#pragma unroll
    for (int i = 0; i < (NBLK + 255) / 256; ++i) {
        const int e = tid + 256 * i, b = e % (C::KW / 8), g = e / (C::KW / 8);
        if (e >= NBLK) break;
        float x[8][8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const float* row = sS + (8 * g + r) * SP + 8 * b;
            const float4 b0 = *reinterpret_cast<const float4*>(row);
            const float4 b1 = *reinterpret_cast<const float4*>(row + 4);
            x[r][0] = b0.x; x[r][1] = b0.y; x[r][2] = b0.z; x[r][3] = b0.w;
            x[r][4] = b1.x; x[r][5] = b1.y; x[r][6] = b1.z; x[r][7] = b1.w;
        }
        v8 hi[8], lo[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) split8<T16>(x[r], hi[r], lo[r]);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            float* row = sS + (8 * g + r) * SP + 8 * b;   // [8 hi][8 lo]
            *reinterpret_cast<v8*>(row) = hi[r];
            *reinterpret_cast<v8*>(row + 4) = lo[r];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int col = 8 * b + c;
            if (col < NC) {
                v8 th, tl;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    th[r] = hi[r][c];
                    tl[r] = lo[r][c];
                }
                const int tr = 16 * (col % CW) + col / CW;   // S^T row of column col
                *reinterpret_cast<v8*>(sTh + tr * TP + 8 * g) = th;
                *reinterpret_cast<v8*>(sTl + tr * TP + 8 * g) = tl;
            }
        }
    }
    __syncthreads();
    // GEMM1 (three products): P[erow + j][16u + lr], K step s2 of 32 with
    // group lk holding k = 32 s2 + 8 lk + i
    f32x4m p[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) p[u] = f32x4m{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const float* blk = sS + (16 * u + lr) * SP + 8 * (4 * s2 + lk);   // [8 hi][8 lo]
            const v8 bh = *reinterpret_cast<const v8*>(blk);
            const v8 bl = *reinterpret_cast<const v8*>(blk + 4);
            p[u] = Mf16<T16>::mma(ah[s2], bh, p[u]);
            p[u] = Mf16<T16>::mma(ah[s2], bl, p[u]);
            p[u] = Mf16<T16>::mma(al[s2], bh, p[u]);
        }
    }
    // E = X_F - P, scaled, rounded to 16 bits into the wavefront's rows;
    // loss estimate from the unrounded residual
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
            sE[(erow + j) * TP + fl] = (T16)(-e * wf);
        }
    }
    __builtin_amdgcn_wave_barrier();   // the residual rows are this wavefront's own
    // GEMM2 (two products), K = 128 samples in steps of 32
    f32x4m acc2[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc2[c] = f32x4m{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s2 = 0; s2 < TF / 32; ++s2) {
        const v8 a = *reinterpret_cast<const v8*>(sE + (16 * w + lr) * TP + 32 * s2 + 8 * lk);
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int off = (16 * c + lr) * TP + 32 * s2 + 8 * lk;
            const v8 bh = *reinterpret_cast<const v8*>(sTh + off);
            const v8 bl = *reinterpret_cast<const v8*>(sTl + off);
            acc2[c] = Mf16<T16>::mma(a, bh, acc2[c]);
            acc2[c] = Mf16<T16>::mma(a, bl, acc2[c]);
        }
    }
    float* out = gpart + (int64_t)sgrp * maxIRR;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = i0 + erow + j;
#pragma unroll
        for (int h = 0; h < CW / 4; ++h) {
            const int col = CW * lr + 4 * h;
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

template <typename T16, typename TX, int CT>
static hipError_t launch_mxw_ct(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx,
                                const float* S, const double* pF, int m, dim3 grid, int groups, int row_tiles,
                                float* gp, double* lp, int maxIRR, hipStream_t st) {
    constexpr size_t shm = MixWideCfg<CT>::lds();
    if (!allow_lds(reinterpret_cast<const void*>(&k_grad_mixed_w<T16, TX, CT>), shm)) return hipErrorInvalidValue;
    const WideModes tab = wide_modes(d, xs, m, sizeof(TX));
    launch_timed(k_grad_mixed_w<T16, TX, CT>, grid, dim3(256), shm, st, d, ms, cores, xs, idx, S, pF, m, groups,
                 row_tiles, gp, lp, maxIRR, wide_rr_fixed(d), tab);
    return hipGetLastError();
}

template <typename T16, typename TX>
static hipError_t launch_mxw_tx(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx,
                                const float* S, const double* pF, int m, dim3 grid, int groups, int row_tiles,
                                float* gp, double* lp, int maxIRR, int maxRR, hipStream_t st) {
    switch ((maxRR + 15) / 16) {
        case 3: return launch_mxw_ct<T16, TX, 3>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 4: return launch_mxw_ct<T16, TX, 4>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 5: return launch_mxw_ct<T16, TX, 5>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 6: return launch_mxw_ct<T16, TX, 6>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 7: return launch_mxw_ct<T16, TX, 7>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        case 8: return launch_mxw_ct<T16, TX, 8>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T16, typename TX, int CT>
static hipError_t launch_mx_ct(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                               const double* pF, int m, dim3 grid, int groups, int row_tiles, float* gp, double* lp,
                               int maxIRR, hipStream_t st) {
    constexpr size_t shm = MixGeom<CT>::lds();
    if (!allow_lds(reinterpret_cast<const void*>(&k_grad_mixed<T16, TX, CT>), shm)) return hipErrorInvalidValue;
    launch_timed(k_grad_mixed<T16, TX, CT>, grid, dim3(256), shm, st, d, ms, cores, xs, idx, S, pF, m, groups,
                 row_tiles, gp, lp, maxIRR);
    return hipGetLastError();
}

template <typename T16, typename TX>
static hipError_t launch_mx_tx(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                               const double* pF, int m, dim3 grid, int groups, int row_tiles, float* gp, double* lp,
                               int maxIRR, int maxRR, hipStream_t st) {
    const int nct = (maxRR + 15) / 16;
#define TRK_MX(C) \
    if (nct <= C) return launch_mx_ct<T16, TX, C>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR, st)
    TRK_MX(1);
    TRK_MX(2);
    TRK_MX(3);
    TRK_MX(4);
    TRK_MX(5);
    TRK_MX(6);
    TRK_MX(7);
    TRK_MX(8);
    TRK_MX(10);
    TRK_MX(12);
    TRK_MX(16);
#undef TRK_MX
    return hipErrorInvalidValue;
}

hipError_t launch_grad_mixed(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, const int32_t* idx, const float* S,
                             const double* pF, int m, int prec, int groups, int row_tiles, float* gp, double* lp,
                             hipStream_t st) {
    const Shape sh = shape_of(d);
    const dim3 grid(xcd_grid(row_tiles, groups));
    const int maxIRR = sh.maxI * sh.maxRR;
    if (wide_applies(d, cores, S, gp, m, groups, sh.maxRR, kWideTF) && (d.x_dtype == TR_F32 || d.x_dtype == TR_F16)) {
        const bool xf = d.x_dtype == TR_F32;
        if (prec == TR_PREC_BF16)
            return xf ? launch_mxw_tx<__bf16, float>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp,
                                                     maxIRR, sh.maxRR, st)
                      : launch_mxw_tx<__bf16, __half>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp,
                                                      lp, maxIRR, sh.maxRR, st);
        if (prec == TR_PREC_F16)
            return xf ? launch_mxw_tx<_Float16, float>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp,
                                                       lp, maxIRR, sh.maxRR, st)
                      : launch_mxw_tx<_Float16, __half>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp,
                                                        lp, maxIRR, sh.maxRR, st);
    }
    if (prec == TR_PREC_BF16) {
        if (d.x_dtype == TR_F32)
            return launch_mx_tx<__bf16, float>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp, maxIRR,
                                               sh.maxRR, st);
        if (d.x_dtype == TR_F16)
            return launch_mx_tx<__bf16, __half>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp,
                                                maxIRR, sh.maxRR, st);
    } else if (prec == TR_PREC_F16) {
        if (d.x_dtype == TR_F32)
            return launch_mx_tx<_Float16, float>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp,
                                                 maxIRR, sh.maxRR, st);
        if (d.x_dtype == TR_F16)
            return launch_mx_tx<_Float16, __half>(d, ms, cores, xs, idx, S, pF, m, grid, groups, row_tiles, gp, lp,
                                                  maxIRR, sh.maxRR, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace trk
