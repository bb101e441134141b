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
#include "internal.hpp"

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
