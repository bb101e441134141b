// a9: full reconstruction X_hat_[1] = G_{1(2)} (G^{!=1}_[2])^T and the RSE of
// Section 4, ||X_hat - X_true||_F / ||X_true||_F, with FP64 sums.
//
// FP32 cores with R_1 R_2 <= 128 take the matrix-core kernel k_recon_mfma:
// a block owns 128 columns j of X_[1] (paper order: column j is the
// multi-index of (i_2..i_N), first fastest), 32 per wavefront.  The block
// builds their subchain rows s_j in LDS (chain products of lateral slices)
// and each wavefront sweeps the rows i_1 of G_{1(2)} in tiles of 32 against
// its 32 rows on the matrix cores.  For the RSE the products are FP16 with a
// hi/lo split (below), the B operand comes pre-packed in lane order (one
// coalesced load per instruction), the 32 x 32 result tile is compared with
// X_true as it leaves the accumulators (each half-wavefront reads 32
// consecutive i_1 of one column, 128 bytes), and X_hat is never stored:
// X_true is read exactly once.  The written reconstruction uses FP32
// products (v_mfma_f32_32x32x2_f32) with B read from G_{1(2)} directly.
//
// Other cases (FP64, larger ranks) take k_recon: every thread takes rows
// i_1 = tid, tid + 256, ... and forms TJ dot products with s_j broadcast
// from LDS.  Per-block FP64 partial sums are added in a fixed order.
#include "internal.hpp"

namespace trk {

constexpr int kReconTJ = 32;
constexpr int kReconCK = 8;

template <typename TC, typename TX, int MODE>   // MODE 0: error sums, 1: write X_hat
__global__ __launch_bounds__(256) void k_recon(tr_desc d, Ptrs cores, const TX* __restrict__ Xt, TX* __restrict__ Xo,
                                               double* __restrict__ part, int want_xx) {
    const int N = d.N;
    const int I0 = d.I[0];
    const int R0 = d.R[0], R1 = d.R[1 % N];
    const int RR = R0 * R1;
    const int RRp = RR + ((RR & 1) ? 0 : 1);
    int64_t J = 1;
    for (int k = 1; k < N; ++k) J *= d.I[k];
    const int64_t j0 = (int64_t)blockIdx.x * kReconTJ;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TC* sS = reinterpret_cast<TC*>(smem_raw);                         // [TJ][RRp]
    int64_t* sOff = reinterpret_cast<int64_t*>(sS + kReconTJ * RRp + 2);   // [TJ]
    const int tid = threadIdx.x;
    // subchain rows of the TJ columns
    for (int e = tid; e < kReconTJ * R1; e += blockDim.x) {
        const int jj = e / R1, s = e % R1;
        const int64_t j = j0 + jj;
        TC* out = sS + jj * RRp + R0 * s;
        if (j >= J) {
            for (int r = 0; r < R0; ++r) out[r] = TC(0);
            if (s == 0) sOff[jj] = 0;
            continue;
        }
        int ik[kMaxOrder];
        int64_t rem = j, off = 0;
        for (int k = 1; k < N; ++k) {
            ik[k] = (int)(rem % d.I[k]);
            rem /= d.I[k];
            off += (int64_t)ik[k] * d.x_stride[k];
        }
        if (s == 0) sOff[jj] = off;
        TC v[kMaxRank];
        {
            const int Rk = d.R[1 % N], Rk1 = d.R[ring_next(1 % N, N)];
            const TC* A = static_cast<const TC*>(cores.p[1 % N]) + (int64_t)ik[1] * Rk * Rk1;
#pragma unroll
            for (int c = 0; c < kMaxRank; ++c) v[c] = c < Rk1 ? A[s + Rk * c] : TC(0);
        }
        for (int k = 2; k < N; ++k) {
            const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
            const TC* A = static_cast<const TC*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
            TC w[kMaxRank];
#pragma unroll
            for (int c = 0; c < kMaxRank; ++c) {
                TC acc = TC(0);
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
        for (int r = 0; r < R0; ++r) out[r] = v[r];
    }
    __syncthreads();
    const TC* G0 = static_cast<const TC*>(cores.p[0]);
    const int64_t xs0 = d.x_stride[0];
    double err = 0.0, xx = 0.0;
    for (int i = tid; i < I0; i += blockDim.x) {
        TC acc[kReconTJ];
#pragma unroll
        for (int jj = 0; jj < kReconTJ; ++jj) acc[jj] = TC(0);
        for (int c0 = 0; c0 < RR; c0 += kReconCK) {
            TC gv[kReconCK];
#pragma unroll
            for (int u = 0; u < kReconCK; ++u) gv[u] = c0 + u < RR ? G0[(int64_t)i * RR + c0 + u] : TC(0);
#pragma unroll
            for (int jj = 0; jj < kReconTJ; ++jj) {
                const TC* sr = sS + jj * RRp + c0;
#pragma unroll
                for (int u = 0; u < kReconCK; ++u)
                    if (c0 + u < RR) acc[jj] += gv[u] * sr[u];
            }
        }
#pragma unroll
        for (int jj = 0; jj < kReconTJ; ++jj) {
            if (j0 + jj < J) {
                const int64_t o = sOff[jj] + (int64_t)i * xs0;
                if (MODE == 0) {
                    const double x = to_f64(Xt[o]);
                    const double df = (double)acc[jj] - x;
                    err += df * df;
                    xx += x * x;
                } else {
                    Xo[o] = from_f64<TX>((double)acc[jj]);
                }
            }
        }
    }
    if (MODE == 0) {
        __shared__ double red[4];
        const double e = block_sum(err, red);
        const double q = block_sum(xx, red);
        if (tid == 0) {
            part[2 * (int64_t)blockIdx.x] = e;
            part[2 * (int64_t)blockIdx.x + 1] = q;
        }
    }
    (void)want_xx;
}

// Fixed-order sum of the per-block partials: strided per thread, then the
// block tree (deterministic for a given block count).
__global__ __launch_bounds__(256) void k_recon_finish(const double* __restrict__ part, int64_t nblocks,
                                                      double xnorm2, double* rse, double* sums) {
    __shared__ double red[4];
    double e = 0.0, q = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
        e += part[2 * b];
        q += part[2 * b + 1];
    }
    e = block_sum(e, red);
    q = block_sum(q, red);
    if (threadIdx.x != 0) return;
    if (xnorm2 >= 0.0) q = xnorm2;
    sums[0] = e;
    sums[1] = q;
    *rse = sqrt(e) / sqrt(q);
}

// ------------------------------------------------------ matrix-core path --

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRmWaves = 4;                 // wavefronts per block
constexpr int kRmCols = 32 * kRmWaves;      // columns j per block

// K steps of two (the B operand's per-lane count) for a given R_1 R_2.
static int recon_kt(int RR) {
    if (RR <= 16) return 8;
    if (RR <= 32) return 16;
    if (RR <= 64) return 32;
    if (RR <= 100) return 50;
    if (RR <= 128) return 64;
    return 0;
}

static bool recon_mfma_ok(const tr_desc& d) {
    return d.core_dtype == TR_F32 && (d.x_dtype == TR_F32 || d.x_dtype == TR_F16) &&
           recon_kt(d.R[0] * d.R[1 % d.N]) > 0;
}

// Error sums on FP16 matrix cores with a hi/lo split (three products per K
// step: lo*hi, hi*lo, hi*hi, FP32 accumulation).  Each operand tile is
// scaled by a power of two that puts its largest magnitude in [2^13, 2^14),
// so hi + lo carries 22 significant bits of every entry that is not far
// below the tile's largest; the result is scaled back exactly.
typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));

__device__ inline int h3_exponent(float mx) {   // mx * 2^e in [2^13, 2^14); 0 if none
    if (!(mx > 0.f) || !(mx <= 3.4e38f)) return 0;
    int x;
    frexpf(mx, &x);
    return 14 - x;
}

// G_{1(2)} split for the B operand of v_mfma_f32_32x32x16_f16, one block per
// row tile it of 32 rows: lane l of K step q holds G(32 it + l % 32,
// 16 q + 8 (l / 32) + i), i < 8, at Bh/Bl[((it K16 + q) 64 + l) 8 + i] (hi and
// lo halves of the scaled value, zero outside); escale[it] is the tile's
// scale exponent.
__global__ __launch_bounds__(256) void k_recon_pack_h3(tr_desc d, const float* __restrict__ G0, int K16,
                                                       _Float16* __restrict__ Bh, _Float16* __restrict__ Bl,
                                                       int* __restrict__ escale) {
    const int I0 = d.I[0], RR = d.R[0] * d.R[1 % d.N];
    const int it = blockIdx.x, tid = threadIdx.x;
    const int per = K16 * 512;          // packed values of the tile
    constexpr int PV = 8 * 512 / 256;   // per thread at K16 = 8
    // every load of the thread in flight together (indices clamped, masked after)
    float v[PV];
    float mx = 0.f;
#pragma unroll
    for (int u = 0; u < PV; ++u) {
        const int p = u * 256 + tid;
        const int q = p >> 9, l = (p >> 3) & 63, i = p & 7;
        const int row = 32 * it + (l & 31), k = 16 * q + 8 * (l >> 5) + i;
        const int rc = row < I0 ? row : I0 - 1, kc = k < RR ? k : RR - 1;
        const float g = G0[(int64_t)rc * RR + kc];
        v[u] = (p < per && row < I0 && k < RR) ? g : 0.f;
        mx = fmaxf(mx, fabsf(v[u]));
    }
    __shared__ float red[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    const int e = h3_exponent(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
#pragma unroll
    for (int u = 0; u < PV; ++u) {
        const int p = u * 256 + tid;
        const float sv = ldexpf(v[u], e);
        const _Float16 h = (_Float16)sv;
        if (p < per) {
            Bh[(int64_t)it * per + p] = h;
            Bl[(int64_t)it * per + p] = (_Float16)(sv - (float)h);
        }
    }
    if (tid == 0) escale[it] = e;
}

// Order 3 builds a block's rows from LDS when its columns touch at most this
// many slices of the last core (true whenever I_2 >= 32).
constexpr int kRmMaxOuter = 8;

// MODE 0: per-block sums of (X_hat - X_true)^2 and X_true^2 into part, on
// the split FP16 products with KT = 8 K16, the B operand from
// k_recon_pack_h3 (Bh, Bl, escale) and the block's subchain rows split into
// hi/lo halves in LDS once they are built.  MODE 1: X_hat written to Xo
// (FP32 products, B operand read from G_{1(2)} directly).
//
// Work split: the block's 128 columns are four column tiles of 32; the
// (row tile, column tile) pairs are taken in row-tile-major order, and each
// wavefront takes a contiguous quarter of them (exactly ceil(I_1/32) pairs
// each), so it loads a B fragment only when its row tile changes.
template <typename TX, int KT, int MODE>
__global__ __launch_bounds__(256) void k_recon_mfma(tr_desc d, Ptrs cores, const TX* __restrict__ Xt,
                                                    TX* __restrict__ Xo, double* __restrict__ part,
                                                    const _Float16* __restrict__ Bh, const _Float16* __restrict__ Bl,
                                                    const int* __restrict__ escale) {
    static_assert(MODE == 1 || KT % 8 == 0, "split products: K in steps of 16");
    constexpr int SP = 2 * KT + 1;          // LDS row pitch of the subchain rows
    const int N = d.N;
    const int I0 = d.I[0];
    const int R0 = d.R[0], R1 = d.R[1 % N];
    const int RR = R0 * R1;
    int64_t J = 1;
    for (int k = 1; k < N; ++k) J *= d.I[k];
    const int64_t j0 = (int64_t)blockIdx.x * kRmCols;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int64_t* sOff = reinterpret_cast<int64_t*>(smem_raw);          // [kRmCols], -1 past J
    float* sS = reinterpret_cast<float*>(sOff + kRmCols);          // [kRmCols][SP]
    float* sP = sS + kRmCols * SP;                                  // order 3: slices of the last core
    const int tid = threadIdx.x;

    // Order 3: column j = i_2 + I_2 i_3 has subchain row M_j = G_2(i_2) G_3(i_3);
    // the block's columns span few i_3, whose slices are staged in LDS, and
    // each item (column, row s of M_j) loads one row of G_2(i_2).
    const int I1 = d.I[1 % N];
    const int64_t jl = (j0 + kRmCols < J ? j0 + kRmCols : J) - 1;
    const int o_lo = N == 3 ? (int)(j0 / I1) : 0;
    const int n_outer = N == 3 && j0 < J ? (int)(jl / I1) - o_lo + 1 : 0;
    const bool staged = N == 3 && n_outer <= kRmMaxOuter;
    if (staged) {
        const int R2 = d.R[2];                       // slices of core 3: R_3 x R_1 (R_{N+1} = R_1)
        const int RR2 = R2 * R0;
        const float* G2 = static_cast<const float*>(cores.p[2]);
        {   // the slices of core 3, all loads of a thread in flight (clamped, masked after)
            constexpr int UB = (kRmMaxOuter * kMaxRR + 255) / 256;
            const int tot = n_outer * RR2;
            float pv[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int e = u * 256 + tid;
                pv[u] = G2[(int64_t)o_lo * RR2 + (e < tot ? e : tot - 1)];
            }
#pragma unroll
            for (int u = 0; u < UB; ++u)
                if (u * 256 + tid < tot) sP[u * 256 + tid] = pv[u];
        }
        // column jj of the block: i_2 = (i2_0 + jj) mod I_2, i_3 = i3_0 + (i2_0 + jj) div I_2 (32-bit)
        const int i2_0 = (int)(j0 % I1), i3_0 = (int)(j0 / I1);
        int* sI2 = reinterpret_cast<int*>(sP + kRmMaxOuter * kMaxRR);   // [kRmCols]
        int* sI3 = sI2 + kRmCols;                                         // [kRmCols], relative to o_lo
        for (int e = tid; e < kRmCols; e += blockDim.x) {
            const int64_t j = j0 + e;
            const int q = (i2_0 + e) / I1;
            const int i2 = i2_0 + e - q * I1, i3 = i3_0 + q;
            sI2[e] = i2;
            sI3[e] = i3 - o_lo;
            sOff[e] = j < J ? (int64_t)i2 * d.x_stride[1] + (int64_t)i3 * d.x_stride[2] : -1;
        }
        __syncthreads();
        const float* G1 = static_cast<const float*>(cores.p[1]);
        const int RR1 = R1 * R2, last = RR1 - 1;
        const int total = kRmCols * R1;
        auto load_row = [&](int e, float (&v)[kMaxRank]) {   // row s of G_2(i_2), clamped in bounds
            const int jj = e / R1, s = e - jj * R1;
            const float* A = G1 + (int64_t)sI2[jj] * RR1;
#pragma unroll
            for (int c = 0; c < kMaxRank; ++c) v[c] = A[min(s + R1 * c, last)];
#pragma unroll
            for (int c = 0; c < kMaxRank; ++c) v[c] = c < R2 ? v[c] : 0.f;   // uniform mask
        };
        float v[kMaxRank];
        if (tid < total) load_row(tid, v);
        for (int e = tid; e < total; e += blockDim.x) {
            float vn[kMaxRank];
            if (e + (int)blockDim.x < total) load_row(e + blockDim.x, vn);   // next item's row in flight
            const int jj = e / R1, s = e - jj * R1;
            const int64_t j = j0 + jj;
            float* out = sS + jj * SP + R0 * s;
            if (j >= J) {
                for (int r = 0; r < R0; ++r) out[r] = 0.f;
            } else {
                // every LDS read of a row issued together: no read behind a
                // branch (entries past R_3 multiply the zeros of v)
                const float* P = sP + sI3[jj] * R2 * R0;
                for (int r = 0; r < R0; ++r) {
                    const float* Pr = P + R2 * r;
                    float acc = 0.f;
#pragma unroll
                    for (int c = 0; c < kMaxRank; ++c) acc += v[c] * Pr[c < R2 ? c : R2 - 1];
                    out[r] = acc;
                }
            }
#pragma unroll
            for (int c = 0; c < kMaxRank; ++c) v[c] = vn[c];
        }
    } else {
        // any order: thread item (column, row s of M_j) through the chain of
        // slice products.  Loads are unconditional (indices clamped into the
        // slice) so that a whole slice row or column is in flight at once;
        // entries past the ranks are masked after the load.
        for (int e = tid; e < kRmCols * R1; e += blockDim.x) {
            const int jj = e / R1, s = e - jj * R1;
            const int64_t j = j0 + jj;
            float* out = sS + jj * SP + R0 * s;
            if (j >= J) {
                for (int r = 0; r < R0; ++r) out[r] = 0.f;
                if (s == 0) sOff[jj] = -1;
                continue;
            }
            int ik[kMaxOrder];
            int64_t rem = j, off = 0;
            for (int k = 1; k < N; ++k) {
                ik[k] = (int)(rem % d.I[k]);
                rem /= d.I[k];
                off += (int64_t)ik[k] * d.x_stride[k];
            }
            if (s == 0) sOff[jj] = off;
            float v[kMaxRank];
            {
                const int Rk = d.R[1 % N], Rk1 = d.R[ring_next(1 % N, N)];
                const float* A = static_cast<const float*>(cores.p[1 % N]) + (int64_t)ik[1] * Rk * Rk1;
                const int last = Rk * Rk1 - 1;
#pragma unroll
                for (int c = 0; c < kMaxRank; ++c) {
                    const float a = A[min(s + Rk * c, last)];
                    v[c] = c < Rk1 ? a : 0.f;
                }
            }
            for (int k = 2; k < N; ++k) {
                const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
                const float* A = static_cast<const float*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
                const int last = Rk * Rk1 - 1;
                float w[kMaxRank];
#pragma unroll
                for (int c = 0; c < kMaxRank; ++c) w[c] = 0.f;
                for (int c = 0; c < Rk1; ++c) {
                    float col[kMaxRank];
#pragma unroll
                    for (int r = 0; r < kMaxRank; ++r) col[r] = A[min(r + Rk * c, last)];
                    float acc = 0.f;
#pragma unroll
                    for (int r = 0; r < kMaxRank; ++r) acc += r < Rk ? v[r] * col[r] : 0.f;
#pragma unroll
                    for (int q = 0; q < kMaxRank; ++q)
                        if (q == c) w[q] = acc;
                }
#pragma unroll
                for (int c = 0; c < kMaxRank; ++c) v[c] = w[c];
            }
            for (int r = 0; r < R0; ++r) out[r] = v[r];
        }
    }
    for (int e = tid; e < kRmCols * (2 * KT - RR); e += blockDim.x) {   // K padding
        const int jj = e / (2 * KT - RR);
        sS[jj * SP + RR + (e - jj * (2 * KT - RR))] = 0.f;
    }
    __syncthreads();

    const int w = tid >> 6, l = tid & 63, lc = l & 31, lh = l >> 5;
    // Result row r of this lane within column tile ct is column
    // 32 ct + 8 (r / 4) + 4 lh + r % 4; its result column is i_1 = 32 it + lc.
    const float* G0 = static_cast<const float*>(cores.p[0]);
    const int64_t xs0 = d.x_stride[0];
    const int nti = (I0 + 31) / 32;
    double err = 0.0, xx = 0.0;
    if constexpr (MODE == 0) {
        // Split the block's rows: every thread reads its share of sS into
        // registers (and its largest magnitude), then, after the block's
        // largest is known and every read is done, writes the hi/lo halves
        // over the same LDS (row pitch HP halves; the FP32 rows, the staged
        // slices and column indices behind them are no longer needed).
        constexpr int K16 = KT / 8, KW = 16 * K16, HP = KW + 8;
        constexpr int PT = kRmCols * KW / 256;   // values per thread
        float v[PT];
        float mx = 0.f;
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int e = u * 256 + tid, row = e / KW, k = e - row * KW;
            v[u] = sS[row * SP + k];
            mx = fmaxf(mx, fabsf(v[u]));
        }
        __shared__ float redm[4];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        if (l == 0) redm[w] = mx;
        __syncthreads();
        const int eA = h3_exponent(fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3])));
        _Float16* Ah = reinterpret_cast<_Float16*>(sS);
        _Float16* Al = Ah + kRmCols * HP;
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int e = u * 256 + tid, row = e / KW, k = e - row * KW;
            const float sv = ldexpf(v[u], eA);
            const _Float16 h = (_Float16)sv;
            Ah[row * HP + k] = h;
            Al[row * HP + k] = (_Float16)(sv - (float)h);
        }
        __syncthreads();
        h16x8 bh[K16], bl[K16];
        int it_loaded = -1;
        double bscale = 0.0;   // 2^-(eA + escale): applied in FP64, exact at any tensor scale
        // X_true entries of pair pr, read at clamped indices and kept as
        // loaded (no select on them, which would wait for the load at
        // once); entries outside the tensor are skipped where they are used
        auto load_x = [&](int pr, TX (&x)[16]) {
            const int it = pr >> 2, ct = pr & 3;
            const int i = 32 * it + lc;
            const int64_t ic = i < I0 ? i : I0 - 1;
            const int64_t* offw = sOff + 32 * ct + 4 * lh;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t o = offw[8 * (r >> 2) + (r & 3)];
                x[r] = Xt[(o >= 0 ? o : 0) + ic * xs0];
            }
        };
        auto pair = [&](int pr, const TX (&x)[16]) {
            const int it = pr >> 2, ct = pr & 3;
            const int i = 32 * it + lc;
            const bool iok = i < I0;
            if (it != it_loaded) {   // B fragment of row tile it, kept across its column tiles
                it_loaded = it;
                const h16x8* sh = reinterpret_cast<const h16x8*>(Bh) + (int64_t)it * K16 * 64 + l;
                const h16x8* sl = reinterpret_cast<const h16x8*>(Bl) + (int64_t)it * K16 * 64 + l;
#pragma unroll
                for (int q = 0; q < K16; ++q) {
                    bh[q] = sh[q * 64];
                    bl[q] = sl[q * 64];
                }
                bscale = ldexp(1.0, -(eA + escale[it]));
            }
            const int64_t* offw = sOff + 32 * ct + 4 * lh;
            const h16x8* ah = reinterpret_cast<const h16x8*>(Ah + (32 * ct + lc) * HP + 8 * lh);
            const h16x8* al = reinterpret_cast<const h16x8*>(Al + (32 * ct + lc) * HP + 8 * lh);
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
            for (int q = 0; q < K16; ++q) {
                const h16x8 a_h = ah[2 * q], a_l = al[2 * q];
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a_l, bh[q], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a_h, bl[q], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a_h, bh[q], acc, 0, 0, 0);
            }
            if (iok) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t o = offw[8 * (r >> 2) + (r & 3)];
                    if (o < 0) continue;
                    const double xd = (double)Cvt<TX>::to_f32(x[r]);
                    const double df = (double)acc[r] * bscale - xd;
                    err += df * df;
                    xx += xd * xd;
                }
            }
        };
        // Two register buffers in turn: the entries of the next pair are
        // requested before this pair's products, so a pair's X_true reads
        // have a whole pair of matrix work to arrive in.
        TX xa[16], xb[16];
        const int pb = w * nti, pe = (w + 1) * nti;
        load_x(pb, xa);
        for (int pr = pb; pr < pe; pr += 2) {
            if (pr + 1 < pe) load_x(pr + 1, xb);
            pair(pr, xa);
            if (pr + 1 < pe) {
                if (pr + 2 < pe) load_x(pr + 2, xa);
                pair(pr + 1, xb);
            }
        }
    } else {
        float b[KT];
        int it_loaded = -1;
        for (int pr = w * nti; pr < (w + 1) * nti; ++pr) {
            const int it = pr >> 2, ct = pr & 3;
            const int i = 32 * it + lc;
            const bool iok = i < I0;
            if (it != it_loaded) {   // B fragment of row tile it, kept across its column tiles
                it_loaded = it;
#pragma unroll
                for (int q = 0; q < KT; ++q) {
                    const int k = 2 * q + lh;
                    b[q] = (iok && k < RR) ? G0[(int64_t)i * RR + k] : 0.f;
                }
            }
            const int64_t* offw = sOff + 32 * ct + 4 * lh;
            const float* arow = sS + (32 * ct + lc) * SP + lh;
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
            for (int q = 0; q < KT; ++q) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(arow[2 * q], b[q], acc, 0, 0, 0);
            if (iok) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t o = offw[8 * (r >> 2) + (r & 3)];
                    if (o >= 0) Xo[o + (int64_t)i * xs0] = from_f64<TX>((double)acc[r]);
                }
            }
        }
    }
    if (MODE == 0) {
        __shared__ double red[4];
        const double e = block_sum(err, red);
        const double q = block_sum(xx, red);
        if (tid == 0) {
            part[2 * (int64_t)blockIdx.x] = e;
            part[2 * (int64_t)blockIdx.x + 1] = q;
        }
    }
}

static size_t recon_mfma_shm(int KT) {
    return (size_t)kRmCols * 8 + (size_t)kRmCols * (2 * KT + 1) * 4 + (size_t)kRmMaxOuter * kMaxRR * 4 +
           (size_t)kRmCols * 8;   // per-column i_2 and i_3 (order 3)
}

static int64_t recon_mfma_blocks(const tr_desc& d) {
    int64_t J = 1;
    for (int k = 1; k < d.N; ++k) J *= d.I[k];
    return (J + kRmCols - 1) / kRmCols;
}

static int recon_k16(const tr_desc& d) { return (d.R[0] * d.R[1 % d.N] + 15) / 16; }

// split B operand: hi and lo halves, then the per-tile scale exponents
static size_t recon_pack_h3_bytes(const tr_desc& d) {
    const size_t nti = (size_t)(d.I[0] + 31) / 32;
    return 2 * align_up(nti * recon_k16(d) * 512 * 2) + align_up(nti * 4);
}

template <typename TX>
static hipError_t launch_recon_write(const tr_desc& d, Ptrs cores, TX* Xo, hipStream_t st) {
    const int KT = recon_kt(d.R[0] * d.R[1 % d.N]);
    const dim3 grid((unsigned)recon_mfma_blocks(d)), block(256);
    const size_t shm = recon_mfma_shm(KT);
#define TRK_RM(KTV)                                                                                      \
    case KTV:                                                                                            \
        if (!allow_lds(reinterpret_cast<const void*>(&k_recon_mfma<TX, KTV, 1>), shm))                  \
            return hipErrorInvalidConfiguration;                                                         \
        hipLaunchKernelGGL((k_recon_mfma<TX, KTV, 1>), grid, block, shm, st, d, cores, (const TX*)nullptr, Xo, \
                           nullptr, nullptr, nullptr, nullptr);                                          \
        break;
    switch (KT) {
        TRK_RM(8)
        TRK_RM(16)
        TRK_RM(32)
        TRK_RM(50)
        TRK_RM(64)
        default:
            return hipErrorInvalidValue;
    }
#undef TRK_RM
    return hipGetLastError();
}

template <typename TX>
static hipError_t launch_recon_h3(const tr_desc& d, Ptrs cores, const _Float16* Bh, const _Float16* Bl,
                                  const int* escale, const TX* Xt, double* part, hipStream_t st) {
    const int K16 = recon_k16(d);
    const dim3 grid((unsigned)recon_mfma_blocks(d)), block(256);
    const size_t shm = recon_mfma_shm(8 * K16);
#define TRK_RH(K)                                                                                         \
    case K:                                                                                               \
        if (!allow_lds(reinterpret_cast<const void*>(&k_recon_mfma<TX, 8 * K, 0>), shm))                 \
            return hipErrorInvalidConfiguration;                                                          \
        hipLaunchKernelGGL((k_recon_mfma<TX, 8 * K, 0>), grid, block, shm, st, d, cores, Xt, (TX*)nullptr, \
                           part, Bh, Bl, escale);                                                         \
        break;
    switch (K16) {
        TRK_RH(1)
        TRK_RH(2)
        TRK_RH(3)
        TRK_RH(4)
        TRK_RH(5)
        TRK_RH(6)
        TRK_RH(7)
        TRK_RH(8)
        default:
            return hipErrorInvalidValue;
    }
#undef TRK_RH
    return hipGetLastError();
}

static size_t recon_shm(const tr_desc& d, size_t es) {
    const int RR = d.R[0] * d.R[1 % d.N];
    const int RRp = RR + ((RR & 1) ? 0 : 1);
    return (size_t)(kReconTJ * RRp + 2) * es + kReconTJ * 8 + 16;
}

static int64_t recon_blocks(const tr_desc& d) {
    int64_t J = 1;
    for (int k = 1; k < d.N; ++k) J *= d.I[k];
    return (J + kReconTJ - 1) / kReconTJ;
}

size_t relerr_ws_bytes(const tr_desc& d) {
    size_t b = align_up(16) + align_up((size_t)recon_blocks(d) * 16);
    if (recon_mfma_ok(d)) b += align_up(recon_pack_h3_bytes(d));
    return b;
}

hipError_t launch_relerr(const tr_desc& d, Ptrs cores, const void* Xt, double xnorm2, double* rse, void* ws,
                         hipStream_t st) {
    char* w = static_cast<char*>(ws);
    double* sums = reinterpret_cast<double*>(w);
    double* part = reinterpret_cast<double*>(w + align_up(16));
    if (recon_mfma_ok(d)) {
        char* pk = w + align_up(16) + align_up((size_t)recon_blocks(d) * 16);
        const int nti = (d.I[0] + 31) / 32, K16 = recon_k16(d);
        const size_t half_bytes = align_up((size_t)nti * K16 * 512 * 2);
        _Float16* Bh = reinterpret_cast<_Float16*>(pk);
        _Float16* Bl = reinterpret_cast<_Float16*>(pk + half_bytes);
        int* escale = reinterpret_cast<int*>(pk + 2 * half_bytes);
        hipLaunchKernelGGL(k_recon_pack_h3, dim3((unsigned)nti), dim3(256), 0, st, d,
                           static_cast<const float*>(cores.p[0]), K16, Bh, Bl, escale);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = d.x_dtype == TR_F32
                ? launch_recon_h3(d, cores, Bh, Bl, escale, static_cast<const float*>(Xt), part, st)
                : launch_recon_h3(d, cores, Bh, Bl, escale, static_cast<const __half*>(Xt), part, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_recon_finish, dim3(1), dim3(256), 0, st, part, recon_mfma_blocks(d), xnorm2, rse,
                           sums);
        return hipGetLastError();
    }
    const int64_t nb = recon_blocks(d);
    const dim3 grid((unsigned)nb);
    const bool f64 = d.core_dtype == TR_F64;
    const size_t shm = recon_shm(d, f64 ? 8 : 4);
    if (f64 && d.x_dtype == TR_F64)
        hipLaunchKernelGGL((k_recon<double, double, 0>), grid, dim3(256), shm, st, d, cores,
                           static_cast<const double*>(Xt), nullptr, part, 1);
    else if (!f64 && d.x_dtype == TR_F32)
        hipLaunchKernelGGL((k_recon<float, float, 0>), grid, dim3(256), shm, st, d, cores,
                           static_cast<const float*>(Xt), nullptr, part, 1);
    else if (!f64 && d.x_dtype == TR_F16)
        hipLaunchKernelGGL((k_recon<float, __half, 0>), grid, dim3(256), shm, st, d, cores,
                           static_cast<const __half*>(Xt), nullptr, part, 1);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_recon_finish, dim3(1), dim3(256), 0, st, part, nb, xnorm2, rse, sums);
    return hipGetLastError();
}

hipError_t launch_reconstruct(const tr_desc& d, Ptrs cores, void* Xo, hipStream_t st) {
    if (recon_mfma_ok(d)) {
        return d.x_dtype == TR_F32 ? launch_recon_write(d, cores, static_cast<float*>(Xo), st)
                                   : launch_recon_write(d, cores, static_cast<__half*>(Xo), st);
    }
    const int64_t nb = recon_blocks(d);
    const dim3 grid((unsigned)nb);
    const bool f64 = d.core_dtype == TR_F64;
    const size_t shm = recon_shm(d, f64 ? 8 : 4);
    if (f64 && d.x_dtype == TR_F64)
        hipLaunchKernelGGL((k_recon<double, double, 1>), grid, dim3(256), shm, st, d, cores, nullptr,
                           static_cast<double*>(Xo), nullptr, 0);
    else if (!f64 && d.x_dtype == TR_F32)
        hipLaunchKernelGGL((k_recon<float, float, 1>), grid, dim3(256), shm, st, d, cores, nullptr,
                           static_cast<float*>(Xo), nullptr, 0);
    else if (!f64 && d.x_dtype == TR_F16)
        hipLaunchKernelGGL((k_recon<float, __half, 1>), grid, dim3(256), shm, st, d, cores, nullptr,
                           static_cast<__half*>(Xo), nullptr, 0);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Mode-major replica: Xn[i + I_n j] = X(i at mode n, column j of X_[n]).
template <typename TX>
__global__ __launch_bounds__(256) void k_replicate(tr_desc d, int n, const TX* __restrict__ X, TX* __restrict__ Xn) {
    const int N = d.N;
    const int In = d.I[n];
    const int64_t J = J_of(d, n);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)In * J) return;
    const int i = (int)(e % In);
    int64_t rem = e / In, off = (int64_t)i * d.x_stride[n];
    int k = ring_next(n, N);
    for (int q = 1; q < N; ++q) {
        off += (rem % d.I[k]) * d.x_stride[k];
        rem /= d.I[k];
        k = ring_next(k, N);
    }
    Xn[e] = X[off];
}

hipError_t launch_replicate(const tr_desc& d, const void* X, int n, void* Xn, hipStream_t st) {
    const int64_t total = (int64_t)d.I[n] * J_of(d, n);
    const dim3 grid((unsigned)((total + 255) / 256));
    switch (d.x_dtype) {
        case TR_F64:
            hipLaunchKernelGGL(k_replicate<double>, grid, dim3(256), 0, st, d, n, static_cast<const double*>(X),
                               static_cast<double*>(Xn));
            break;
        case TR_F32:
            hipLaunchKernelGGL(k_replicate<float>, grid, dim3(256), 0, st, d, n, static_cast<const float*>(X),
                               static_cast<float*>(Xn));
            break;
        default:
            hipLaunchKernelGGL(k_replicate<uint16_t>, grid, dim3(256), 0, st, d, n, static_cast<const uint16_t*>(X),
                               static_cast<uint16_t*>(Xn));
            break;
    }
    return hipGetLastError();
}

}  // namespace trk
