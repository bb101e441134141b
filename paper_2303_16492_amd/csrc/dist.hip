// a2: the sampling laws of Section 3.2 turned into integer-weight CDFs.
//
//   Euclidean (Lemma euc_est): p(i) = ||G_k(:,i,:)||_F^2 / ||G_k||_F^2.
//   Leverage (Lemma lev_est):  p(i) = l_i(G_{k(2)}) / rank, l_i = g_i^T (G^T G)^{-1} g_i
//                              with the FP64 Gram G^T G of G = G_{k(2)} (the sweep
//                              inverse for R_k R_{k+1} <= 128, ||L^{-1} g_i||^2 with
//                              its Cholesky factor L above); a Gram that is singular
//                              or close to it, and I_k <= R_k R_{k+1}, take the
//                              rank-revealing route (pivoted Cholesky, scores on the
//                              chosen columns, divided by the rank found).
//   Optimal (eq:optimal_prob): q(j) ~ ||X_[n](:,j) - G_{n(2)} s_j|| * ||s_j||
//                              over the J_n columns, FP64.
// Weights w = floor(p 2^40) + 1 and their inclusive prefix sums are exact
// integers: the sampler's choice depends only on them.
#include "internal.hpp"

namespace trk {

constexpr double kTwo40 = 1099511627776.0;

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Inclusive scan of a[0..len) (uint64) by one block, in place: each thread
// scans a contiguous segment, the segment sums are scanned across lanes with
// shuffles and across wavefronts through LDS, and each segment adds its
// offset.  Integer sums: the result does not depend on the grouping.
__device__ inline void block_scan_u64(uint64_t* a, int64_t len) {
    __shared__ uint64_t wtot[16];
    const int T = blockDim.x, lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (T + 63) >> 6;
    const int64_t per = (len + T - 1) / T;
    const int64_t b = threadIdx.x * per, e = min(len, b + per);
    uint64_t s = 0;
    for (int64_t i = b; i < e; ++i) {
        s += a[i];
        a[i] = s;
    }
    uint64_t incl = s;   // inclusive scan of the segment sums within the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(incl, (unsigned)o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wid] = incl;
    __syncthreads();
    if (wid == 0) {   // exclusive scan of the wavefront totals
        const uint64_t v = lane < nw ? wtot[lane] : 0ull;
        uint64_t x = v;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const uint64_t y = __shfl_up(x, (unsigned)o, 64);
            if (lane >= o) x += y;
        }
        if (lane < nw) wtot[lane] = x - v;
    }
    __syncthreads();
    const uint64_t off = wtot[wid] + incl - s;
    for (int64_t i = b; i < e; ++i) a[i] += off;
    __syncthreads();
}

__device__ inline uint64_t quantize(double p) { return (uint64_t)floor(p * kTwo40) + 1ull; }

__device__ inline void write_uniform_weights(uint64_t* w, int64_t len) {
    const uint64_t wu = quantize(1.0 / (double)len);
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) w[i] = wu;
    __syncthreads();
}

// Weights staged in LDS when every core has at most this many rows (the
// launch then passes lds_rows = max I_k, else 0).
constexpr int kLdsRows = 8192;
constexpr int kLevLdsRows = 4096;

// w (Ik weights, in LDS or global memory) -> inclusive CDF in cdf; the
// step counter advances afterwards when ``bump`` is set (every thread of
// the block read it before the block's first barrier).
__device__ inline void finish_cdf(uint64_t* w, uint64_t* cdf, int Ik, uint64_t* bump) {
    block_scan_u64(w, Ik);
    if (w != cdf)
        for (int i = threadIdx.x; i < Ik; i += blockDim.x) cdf[i] = w[i];
    if (bump && threadIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long*>(bump), 1ull);
}

// Euclidean law of core k in two launches: the row norms ||g_i||^2 across
// the GPU (a wavefront takes four rows, its lanes across the row, coalesced,
// at most four passes of 64 since RR <= 256, then a shuffle sum), then the
// total, weights, CDF and (inside a step) the counter advance in one block.
constexpr int kEucRows = 16;

template <typename TC>
__global__ __launch_bounds__(256) void k_euc_rows(tr_desc d, ModeSrc ms, int use_mode, int k_fixed, Ptrs cores,
                                                  double* __restrict__ rn) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    const int RR = d.R[k] * d.R[ring_next(k, d.N)];
    const int i0 = blockIdx.x * kEucRows + 4 * (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i0 >= Ik) return;
    const TC* G = static_cast<const TC*>(cores.p[k]);
    double s[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + r < Ik ? i0 + r : Ik - 1;
        s[r] = 0.0;
#pragma unroll
        for (int pa = 0; pa < 4; ++pa) {
            const int c = lane + 64 * pa;
            const double v = (double)G[(int64_t)i * RR + (c < RR ? c : RR - 1)];
            s[r] += c < RR ? v * v : 0.0;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double tr = wave_sum(s[r]);
        if (lane == 0 && i0 + r < Ik) rn[i0 + r] = tr;
    }
}

__global__ __launch_bounds__(1024) void k_euc_cdf(tr_desc d, ModeSrc ms, int use_mode, int k_fixed,
                                                  const double* __restrict__ rn, MutPtrs cdf_out, int32_t* status,
                                                  uint64_t* bump, int lds_rows) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    uint64_t* cdf = static_cast<uint64_t*>(cdf_out.p[k]);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint64_t* w = Ik <= lds_rows ? reinterpret_cast<uint64_t*>(smem_raw) : cdf;
    double loc = 0.0;
    for (int i = threadIdx.x; i < Ik; i += blockDim.x) loc += rn[i];
    __shared__ double red[16];
    const double tot = block_sum(loc, red);
    if (!(tot > 0.0) || !isfinite(tot)) {
        if (threadIdx.x == 0) set_status(status, TR_DEV_ZERO_DIST);
        write_uniform_weights(w, Ik);
    } else {
        for (int i = threadIdx.x; i < Ik; i += blockDim.x) w[i] = quantize(rn[i] / tot);
        __syncthreads();
    }
    finish_cdf(w, cdf, Ik, bump);
}

// ----------------------------------------------------- rank-revealing law --
//
// Leverage law of a core whose unfolding may be rank deficient (Lemma
// lev_est divides the scores of Definition "Leverage Scores" by the rank):
// Cholesky with diagonal pivoting on the Gram B = G^T G of G = G_{k(2)}
// (the largest remaining pivot first), stopped once no remaining pivot
// exceeds RR 2^-52 max_i B_ii; r = the steps taken is the rank.  The chosen
// columns P of G span its column space, so with L the r x r factor of B_PP
//     l_i = g_i[P]^T (G_P^T G_P)^{-1} g_i[P] = ||L^{-1} g_i[P]||^2,
// and r = I_k (full row rank, possible only when I_k <= RR) gives l_i = 1.
// One block of 1024 threads.  Bm: RR x RR doubles of device scratch
// (row-major) holding G^T G on entry, overwritten.  Writes the weights
// floor(l_i / r 2^40) + 1 into w (r = 0, a zero core: the uniform law and
// TR_DEV_ZERO_DIST).
// Pivot test that sends the fast path here: 2^-43 of the largest diagonal
// entry, a few times the rounding of a Gram summed over a few hundred rows
// (so a pivot of a dependent column is caught) while an ill-conditioned core
// of full rank (sigma_min / sigma_max above about 3.4e-7) stays on the fast
// path; both Gram routes carry the same kappa^2 u error on such a core.
constexpr double kLevTrigger = 1.0 / 8796093022208.0;

template <typename TC>
__device__ void leverage_pivoted(const TC* __restrict__ G, int Ik, int RR, double* __restrict__ Bm,
                                 uint64_t* __restrict__ w, int32_t* status) {
    __shared__ int perm[kMaxRR];
    __shared__ double dinv[kMaxRR];
    __shared__ double xw[8][kMaxRR];   // rows are scored by the first eight wavefronts
    __shared__ double rv[16];
    __shared__ int ri[16];
    __shared__ double red[16];
    const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = T >> 6;
    const int nB = RR;
    for (int i = tid; i < nB; i += T) perm[i] = i;
    __syncthreads();
    double mx = 0.0;
    for (int i = tid; i < nB; i += T) mx = fmax(mx, Bm[(int64_t)i * nB + i]);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) red[wid] = mx;
    __syncthreads();
    mx = 0.0;
    for (int q = 0; q < nw; ++q) mx = fmax(mx, red[q]);
    const double tol = (double)nB * 2.220446049250313e-16 * mx;
    int r = 0;
    for (int j = 0; j < nB; ++j) {
        // largest remaining pivot (ties: the smallest index)
        double bv = -1.0;
        int bi = nB;
        for (int i = j + tid; i < nB; i += T) {
            const double v = Bm[(int64_t)i * nB + i];
            if (v > bv) { bv = v; bi = i; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { rv[wid] = bv; ri[wid] = bi; }
        __syncthreads();
        bv = rv[0];
        bi = ri[0];
        for (int q = 1; q < nw; ++q)
            if (rv[q] > bv || (rv[q] == bv && ri[q] < bi)) { bv = rv[q]; bi = ri[q]; }
        __syncthreads();
        if (!(bv > tol) || !isfinite(bv)) break;   // the same verdict in every thread
        r = j + 1;
        if (bi != j) {   // symmetric exchange of j and bi: rows (all columns), then columns of the trailing rows
            for (int c = tid; c < nB; c += T) {
                const double a = Bm[(int64_t)j * nB + c];
                Bm[(int64_t)j * nB + c] = Bm[(int64_t)bi * nB + c];
                Bm[(int64_t)bi * nB + c] = a;
            }
            __syncthreads();
            for (int i = j + tid; i < nB; i += T) {
                const double a = Bm[(int64_t)i * nB + j];
                Bm[(int64_t)i * nB + j] = Bm[(int64_t)i * nB + bi];
                Bm[(int64_t)i * nB + bi] = a;
            }
            if (tid == 0) {
                const int a = perm[j];
                perm[j] = perm[bi];
                perm[bi] = a;
            }
            __syncthreads();
        }
        const double ljj = sqrt(Bm[(int64_t)j * nB + j]);
        __syncthreads();
        for (int i = j + 1 + tid; i < nB; i += T) Bm[(int64_t)i * nB + j] /= ljj;
        if (tid == 0) Bm[(int64_t)j * nB + j] = ljj;
        __syncthreads();
        const int wd = nB - j - 1;
        for (int e = tid; e < wd * wd; e += T) {
            const int i = j + 1 + e / wd, c = j + 1 + e % wd;
            Bm[(int64_t)i * nB + c] -= Bm[(int64_t)i * nB + j] * Bm[(int64_t)c * nB + j];
        }
        __syncthreads();
    }
    if (r == 0 || r == Ik) {   // zero core, or full row rank: every score 0 or 1
        if (r == 0 && tid == 0) set_status(status, TR_DEV_ZERO_DIST);
        write_uniform_weights(w, Ik);
        return;
    }
    // L^{-1}: column c by thread c; its diagonal in dinv, the rest in the
    // free upper triangle (entry (jj, c) of L^{-1} at Bm[c][jj]).
    for (int c = tid; c < r; c += T) {
        const double yc = 1.0 / Bm[(int64_t)c * nB + c];
        dinv[c] = yc;
        for (int jj = c + 1; jj < r; ++jj) {
            double acc = Bm[(int64_t)jj * nB + c] * yc;
            for (int k = c + 1; k < jj; ++k) acc += Bm[(int64_t)jj * nB + k] * Bm[(int64_t)c * nB + k];
            Bm[(int64_t)c * nB + jj] = -acc / Bm[(int64_t)jj * nB + jj];
        }
    }
    __syncthreads();
    // l_i, one row per wavefront: x = g_i[P] staged in LDS, then z = L^{-1} x
    // with the lanes over the entries of z.
    double* x = xw[wid & 7];
    for (int i = wid; i < Ik && wid < 8; i += 8) {
        for (int c = lane; c < r; c += 64) x[c] = (double)G[(int64_t)i * RR + perm[c]];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double acc = 0.0;
        for (int jj = lane; jj < r; jj += 64) {
            double z = dinv[jj] * x[jj];
            for (int c = 0; c < jj; ++c) z += Bm[(int64_t)c * nB + jj] * x[c];
            acc += z * z;
        }
        acc = wave_sum(acc);
        if (lane == 0) w[i] = quantize(acc / (double)r);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
}

// Leverage law of core k (one block): Gram, Cholesky, row solves.
template <typename TC>
__global__ __launch_bounds__(1024) void k_dist_leverage(tr_desc d, ModeSrc ms, int use_mode, int k_fixed,
                                                        Ptrs cores, MutPtrs cdf_out, int32_t* status,
                                                        double* __restrict__ A, uint64_t* bump) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    const int RR = d.R[k] * d.R[ring_next(k, d.N)];
    const TC* G = static_cast<const TC*>(cores.p[k]);
    uint64_t* w = static_cast<uint64_t*>(cdf_out.p[k]);
    double* lev = reinterpret_cast<double*>(w);
    for (int e = threadIdx.x; e < RR * RR; e += blockDim.x) {
        const int a = e % RR, b = e / RR;
        double s = 0.0;
        for (int i = 0; i < Ik; ++i) s += (double)G[(int64_t)i * RR + a] * (double)G[(int64_t)i * RR + b];
        A[e] = s;
    }
    __syncthreads();
    if (Ik <= RR) {   // the Gram is singular: pivoted; full row rank gives the uniform law
        leverage_pivoted(G, Ik, RR, A, w, status);
        finish_cdf(w, w, Ik, bump);
        return;
    }
    __shared__ double dmax[16];
    double mx = 0.0;
    for (int c = threadIdx.x; c < RR; c += blockDim.x) mx = fmax(mx, A[c + (int64_t)RR * c]);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) dmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) mx = fmax(mx, dmax[q]);
    const double ptol = kLevTrigger * mx;
    // Right-looking Cholesky in A (column-major); a pivot at or below ptol
    // sends the law to the rank-revealing route.
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    for (int j = 0; j < RR; ++j) {
        __syncthreads();
        const double djj = A[j + (int64_t)RR * j];
        if (!(djj > ptol) || !isfinite(djj)) {
            if (threadIdx.x == 0) bad = 1;
            break;
        }
        const double ljj = sqrt(djj);
        __syncthreads();
        for (int i = j + threadIdx.x; i < RR; i += blockDim.x)
            A[i + (int64_t)RR * j] = i == j ? ljj : A[i + (int64_t)RR * j] / ljj;
        __syncthreads();
        const int wd = RR - j - 1;
        for (int e = threadIdx.x; e < wd * wd; e += blockDim.x) {
            const int i = j + 1 + e % wd, c = j + 1 + e / wd;
            if (c <= i) A[i + (int64_t)RR * c] -= A[i + (int64_t)RR * j] * A[c + (int64_t)RR * j];
        }
    }
    __syncthreads();
    if (bad) {   // rank deficient (or close to it): the Gram again, then pivoted
        for (int e = threadIdx.x; e < RR * RR; e += blockDim.x) {
            const int a = e % RR, b = e / RR;
            double s = 0.0;
            for (int i = 0; i < Ik; ++i) s += (double)G[(int64_t)i * RR + a] * (double)G[(int64_t)i * RR + b];
            A[e] = s;
        }
        __syncthreads();
        leverage_pivoted(G, Ik, RR, A, w, status);
        finish_cdf(w, w, Ik, bump);
        return;
    }
    // l_i = ||L^{-1} g_i||^2 by forward substitution, one row per thread.
    for (int i = threadIdx.x; i < Ik; i += blockDim.x) {
        double z[kMaxRR];
        double s = 0.0;
        for (int j = 0; j < RR; ++j) {
            double v = (double)G[(int64_t)i * RR + j];
            for (int c = 0; c < j; ++c) v -= A[j + (int64_t)RR * c] * z[c];
            v /= A[j + (int64_t)RR * j];
            z[j] = v;
            s += v * v;
        }
        lev[i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Ik; i += blockDim.x) w[i] = quantize(lev[i] / (double)RR);
    __syncthreads();
    finish_cdf(w, w, Ik, bump);
}

// The same law for R_k R_{k+1} <= 128 with the factor kept in LDS (one
// block of 1024 threads): (1) the lower triangle of A = G^T G, rows of G
// staged through LDS in chunks, every entry summed over i ascending; (2)
// right-looking Cholesky A = L L^T; (3) L^{-1} in place, column by column
// from the last (column j below the diagonal is -(1/L_jj) L22^{-1} L(j+1:, j)
// with L22^{-1} already formed); (4) l_i = ||L^{-1} g_i||^2, the rows of G
// staged again, each row's RR entries of L^{-1} g_i split over a group of
// threads and their squares summed by a shuffle reduction.
// Leverage law for R_k R_{k+1} <= 128 in four launches across the GPU: the
// FP64 Gram of G_{k(2)} (the sampled-Gram kernels on the core's own rows),
// -(G^T G)^{-1} by the one-workgroup sweep, then
//     l_i = g_i^T (G^T G)^{-1} g_i = -g_i . (g_i (-(G^T G)^{-1}))
// for every row on the FP64 matrix cores, then the weights, CDF and
// (inside a step) the counter advance in one block.

constexpr int kLevRows = 16;

// l_i for 16 rows per block: wavefront w owns output columns 16 n.., n = w
// and w + 4 (K = RR <= 128 in steps of 4), each lane's partial dot products
// are added across its 16 lanes, then across the four wavefronts in a fixed
// order.  Loads at clamped indices, masked afterwards.
template <typename TC>
__global__ __launch_bounds__(256) void k_lev_rows(tr_desc d, ModeSrc ms, int use_mode, int k_fixed, Ptrs cores,
                                                  const double* __restrict__ hm, double* __restrict__ lev) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    const int RR = d.R[k] * d.R[ring_next(k, d.N)];
    const int r0 = blockIdx.x * kLevRows;
    if (r0 >= Ik) return;
    const TC* G = static_cast<const TC*>(cores.p[k]);
    const int tid = threadIdx.x, l = tid & 63, lr = l & 15, lk = l >> 4, w = tid >> 6;
    constexpr int KS = 32;
    const int row = r0 + lr, rowc = row < Ik ? row : Ik - 1;
    TC ga[KS];
    double hb[2][KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int kk = 4 * ks + lk, kc = kk < RR ? kk : RR - 1;
        if (4 * ks < RR) {   // uniform
            ga[ks] = G[(int64_t)rowc * RR + kc];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int c = 16 * (w + 4 * u) + lr, cc = c < RR ? c : RR - 1;
                hb[u][ks] = hm[(int64_t)kc * RR + cc];
            }
        }
    }
    TC gd[2][4];   // G[r0 + 4 j + lk][c], the entries this lane's outputs pair with
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * j + lk, rc = r < Ik ? r : Ik - 1;
            const int c = 16 * (w + 4 * u) + lr, cc = c < RR ? c : RR - 1;
            gd[u][j] = G[(int64_t)rc * RR + cc];
        }
    double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = 16 * (w + 4 * u) + lr;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            if (4 * ks < RR) {
                const int kk = 4 * ks + lk;
                const double a = (row < Ik && kk < RR) ? (double)ga[ks] : 0.0;
                const double b = (kk < RR && c < RR) ? hb[u][ks] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] += c < RR ? (double)gd[u][j] * acc[j] : 0.0;
    }
    __shared__ double sp[4][kLevRows];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double v = part[j];
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);   // the 16 lanes of one row
        if (lr == 0) sp[w][4 * j + lk] = v;
    }
    __syncthreads();
    if (tid < kLevRows && r0 + tid < Ik)
        lev[r0 + tid] = -(((sp[0][tid] + sp[1][tid]) + sp[2][tid]) + sp[3][tid]);
}

// Weights floor(l_i / RR 2^40) + 1 and their CDF (one block).  When the
// sweep found a pivot at or below 2^-43 max_i h_ii (the Gram is singular or
// close to it), or when I_k <= RR, the scores come from the rank-revealing
// route instead (it overwrites the Gram ``gram``).
template <typename TC>
__global__ __launch_bounds__(1024) void k_lev_cdf(tr_desc d, ModeSrc ms, int use_mode, int k_fixed, Ptrs cores,
                                                  double* __restrict__ gram, const double* __restrict__ lev,
                                                  const int* __restrict__ flag, MutPtrs cdf_out, int32_t* status,
                                                  uint64_t* bump, int lds_rows) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    const int RR = d.R[k] * d.R[ring_next(k, d.N)];
    uint64_t* cdf = static_cast<uint64_t*>(cdf_out.p[k]);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint64_t* w = Ik <= lds_rows ? reinterpret_cast<uint64_t*>(smem_raw) : cdf;
    if (Ik <= RR || *flag != 0) {
        leverage_pivoted(static_cast<const TC*>(cores.p[k]), Ik, RR, gram, w, status);
    } else {
        for (int i = threadIdx.x; i < Ik; i += blockDim.x) w[i] = quantize(lev[i] / (double)RR);
        __syncthreads();
    }
    finish_cdf(w, cdf, Ik, bump);
}

struct LevWs {
    GramWs g;
    size_t gram_off, upd_off, lev_off, total;
    UpdWs u;
};

static LevWs lev_ws_layout(const tr_desc& d) {
    const Shape sh = shape_of(d);
    LevWs L{};
    L.g = gram_ws_layout(d, sh.maxI);
    L.gram_off = L.g.total;
    L.upd_off = L.gram_off + align_up((size_t)sh.maxRR * sh.maxRR * 8);
    L.u = UpdWs{};
    L.u.L_off = 0;
    L.u.flag_off = align_up((size_t)sh.maxRR * sh.maxRR * 8);
    L.u.total = L.u.flag_off + 256;
    L.lev_off = L.upd_off + L.u.total;
    L.total = L.lev_off + align_up((size_t)sh.maxI * 8);
    return L;
}

size_t dist_ws_bytes(const tr_desc& d, int law) {
    const Shape sh = shape_of(d);
    if (law == TR_LAW_EUCLID) return align_up((size_t)sh.maxI * 8);   // row norms
    if (law != TR_LAW_LEVERAGE) return 256;
    return sh.maxRR <= 128 ? lev_ws_layout(d).total : align_up((size_t)sh.maxRR * sh.maxRR * 8);
}

hipError_t launch_dist(const tr_desc& d, ModeSrc ms, bool use_mode, int k, int law, Ptrs cores,
                       uint64_t* const* cdf_out, int32_t* status, void* ws, hipStream_t st, uint64_t* bump) {
    MutPtrs out{};
    for (int q = 0; q < d.N; ++q) out.p[q] = cdf_out[q];
    const bool f64 = d.core_dtype == TR_F64;
    const Shape sh = shape_of(d);
    const int lds_rows = sh.maxI <= kLdsRows ? sh.maxI : 0;
    const size_t lds = (size_t)lds_rows * 8;
    if (law == TR_LAW_EUCLID) {
        double* rn = static_cast<double*>(ws);
        const dim3 grid((sh.maxI + kEucRows - 1) / kEucRows);
        if (f64)
            hipLaunchKernelGGL(k_euc_rows<double>, grid, dim3(256), 0, st, d, ms, (int)use_mode, k, cores, rn);
        else
            hipLaunchKernelGGL(k_euc_rows<float>, grid, dim3(256), 0, st, d, ms, (int)use_mode, k, cores, rn);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_euc_cdf, dim3(1), dim3(1024), lds, st, d, ms, (int)use_mode, k, rn, out, status, bump,
                           lds_rows);
    } else if (law == TR_LAW_LEVERAGE && sh.maxRR <= 128) {
        // the mode source of the Gram, the inverse and the scores: the step's
        // mode, or core k
        const ModeSrc mk = use_mode ? ms : ModeSrc{nullptr, 0, k, 0};
        const LevWs L = lev_ws_layout(d);
        char* w = static_cast<char*>(ws);
        double* gram = reinterpret_cast<double*>(w + L.gram_off);
        hipError_t e = launch_gram(d, mk, nullptr, nullptr, sh.maxI, gram, w, L.g, st, nullptr, cores);
        if (e != hipSuccess) return e;
        // no status from the inverse and no damping ladder: a pivot at or
        // below 2^-43 of the largest diagonal entry sends the CDF kernel to
        // the rank-revealing route
        e = launch_sweep_inverse(d, mk, gram, 0.0, L.u, w + L.upd_off, nullptr, st, kLevTrigger);
        if (e != hipSuccess) return e;
        const double* hm = reinterpret_cast<const double*>(w + L.upd_off + L.u.L_off);
        const int* flag = reinterpret_cast<const int*>(w + L.upd_off + L.u.flag_off);
        double* lev = reinterpret_cast<double*>(w + L.lev_off);
        const dim3 grid((sh.maxI + kLevRows - 1) / kLevRows);
        // the CDF kernel's static LDS (rank-revealing route, about 20 KB)
        // plus the staged weights stay within 64 KB
        const int lev_lds_rows = sh.maxI <= kLevLdsRows ? sh.maxI : 0;
        const size_t lev_lds = (size_t)lev_lds_rows * 8;
        if (f64)
            hipLaunchKernelGGL(k_lev_rows<double>, grid, dim3(256), 0, st, d, ms, (int)use_mode, k, cores, hm, lev);
        else
            hipLaunchKernelGGL(k_lev_rows<float>, grid, dim3(256), 0, st, d, ms, (int)use_mode, k, cores, hm, lev);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (f64)
            hipLaunchKernelGGL(k_lev_cdf<double>, dim3(1), dim3(1024), lev_lds, st, d, ms, (int)use_mode, k, cores,
                               gram, lev, flag, out, status, bump, lev_lds_rows);
        else
            hipLaunchKernelGGL(k_lev_cdf<float>, dim3(1), dim3(1024), lev_lds, st, d, ms, (int)use_mode, k, cores,
                               gram, lev, flag, out, status, bump, lev_lds_rows);
    } else if (law == TR_LAW_LEVERAGE) {
        double* A = static_cast<double*>(ws);
        if (f64)
            hipLaunchKernelGGL(k_dist_leverage<double>, dim3(1), dim3(1024), 0, st, d, ms, (int)use_mode, k,
                               cores, out, status, A, bump);
        else
            hipLaunchKernelGGL(k_dist_leverage<float>, dim3(1), dim3(1024), 0, st, d, ms, (int)use_mode, k,
                               cores, out, status, A, bump);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- optimal --

constexpr int kOptBlock = 256;

// a_j = ||X_[n](:,j) - G_{n(2)} s_j||_2 * ||s_j||_2 in FP64, one thread per column.
template <typename TC, typename TX>
__global__ __launch_bounds__(kOptBlock) void k_opt_terms(tr_desc d, ModeSrc ms, Ptrs cores, XSrc xs,
                                                        double* __restrict__ a) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    n = __builtin_amdgcn_readfirstlane(n);   // uniform: its table reads stay scalar
    const int N = d.N;
    const int n1 = ring_next(n, N);
    const int Rn = d.R[n], Rn1 = d.R[n1];
    const int RR = Rn * Rn1;
    const int64_t J = J_of(d, n);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    int ik[kMaxOrder];
    int64_t rem = j, off = 0;
    {
        int k = n1;
        for (int q = 1; q < N; ++q) {
            ik[k] = (int)(rem % d.I[k]);
            rem /= d.I[k];
            off += (int64_t)ik[k] * d.x_stride[k];
            k = ring_next(k, N);
        }
    }
    // s_j (row-major in (s, r): s_j[r + Rn s] = M(s, r)), M built row by row.
    double sj[kMaxRR];
    for (int s = 0; s < Rn1; ++s) {
        double v[kMaxRank];
        int k = n1;
        {
            const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
            const TC* A = static_cast<const TC*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
            for (int c = 0; c < Rk1; ++c) v[c] = (double)A[s + Rk * c];
        }
        for (int q = 2; q < N; ++q) {
            k = ring_next(k, N);
            const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
            const TC* A = static_cast<const TC*>(cores.p[k]) + (int64_t)ik[k] * Rk * Rk1;
            double wv[kMaxRank];
            for (int c = 0; c < Rk1; ++c) {
                double acc = 0.0;
                for (int r = 0; r < Rk; ++r) acc += v[r] * (double)A[r + Rk * c];
                wv[c] = acc;
            }
            for (int c = 0; c < Rk1; ++c) v[c] = wv[c];
        }
        for (int r = 0; r < Rn; ++r) sj[r + Rn * s] = v[r];
    }
    double ss = 0.0;
    for (int c = 0; c < RR; ++c) ss += sj[c] * sj[c];
    const TC* Gn = static_cast<const TC*>(cores.p[n]);
    const TX* X = static_cast<const TX*>(xs.X);
    const int64_t xsn = d.x_stride[n];
    double rr = 0.0;
    for (int i = 0; i < d.I[n]; ++i) {
        double pred = 0.0;
        for (int c = 0; c < RR; ++c) pred += (double)Gn[(int64_t)i * RR + c] * sj[c];
        const double r = to_f64(X[off + (int64_t)i * xsn]) - pred;
        rr += r * r;
    }
    a[j] = sqrt(rr) * sqrt(ss);
}

// The same terms read from the mode-major replica of X, where the fiber
// X_[n](:,j) is contiguous at j I_n (columns in the ring order n+1, n+2, ...
// with the first fastest, as above).  A block takes kOptCols consecutive
// columns.  It forms s_j of every column in LDS (one thread per (column,
// row s of the chain product), the slices read from the cores in global
// memory, which stay in cache), and each wavefront then takes kOptCols / 4
// consecutive columns:
// the predictions G_{n(2)} s_j of its 16 columns are 16 x 16 tiles of FP64
// matrix-core products (its fiber entries requested, in the products'
// result layout, before any arithmetic), and the squared residuals of a
// column are added over its rows in a fixed order.  Needs I_n <= 64 Q,
// R_n R_{n+1} <= kOptRRMax, every rank <= kOptRank and J_n < 2^31.  (At the
// order-4 workload, staging the other cores in LDS measured the same, 98 us;
// all N cores 120 us and G_{n(2)} alone 102 us.)
constexpr int kOptCols = 64;
constexpr int kOptRRMax = 32;
constexpr int kOptRank = 8;                   // every R_k

template <typename TC, typename TX, int Q>
__global__ __launch_bounds__(256) void k_opt_terms_rep(tr_desc d, ModeSrc ms, Ptrs cores, XSrc xs,
                                                       double* __restrict__ a) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    n = __builtin_amdgcn_readfirstlane(n);   // uniform: its table reads stay scalar
    const int N = d.N;
    const int n1 = ring_next(n, N);
    const int Rn = d.R[n], Rn1 = d.R[n1];
    const int RR = Rn * Rn1, In = d.I[n];
    const int64_t J = J_of(d, n);
    const int64_t j0 = (int64_t)blockIdx.x * kOptCols;
    if (j0 >= J) return;   // the whole block
    __shared__ double sS[kOptCols][kOptRRMax + 1];
    __shared__ double sN[kOptCols];
    const int tid = threadIdx.x;
    for (int e = tid; e < kOptCols * (kOptRRMax + 1); e += 256) (&sS[0][0])[e] = 0.0;
    __syncthreads();
    // Row s of the chain product of column j: the slices of cores n+1, ...,
    // n-1 at the column's indices (decoded in that order, the first
    // fastest), every loop bounded by kOptRank at compile time so that the
    // row stays in registers and a stage's LDS reads issue together.
    for (int w = tid; w < kOptCols * Rn1; w += 256) {
        const int c = w / Rn1, s = w - c * Rn1;
        if (j0 + c >= J) continue;
        uint32_t rem = (uint32_t)(j0 + c);
        int k = n1;
        int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
        uint32_t ik = rem % (uint32_t)d.I[k];
        rem /= (uint32_t)d.I[k];
        const TC* A = static_cast<const TC*>(cores.p[k]) + ik * Rk * Rk1;
        double v[kOptRank];
#pragma unroll
        for (int cc = 0; cc < kOptRank; ++cc) v[cc] = cc < Rk1 ? (double)A[s + Rk * cc] : 0.0;
        for (int q = 2; q < N; ++q) {
            k = ring_next(k, N);
            Rk = d.R[k];
            Rk1 = d.R[ring_next(k, N)];
            ik = rem % (uint32_t)d.I[k];
            rem /= (uint32_t)d.I[k];
            A = static_cast<const TC*>(cores.p[k]) + ik * Rk * Rk1;
            double nv[kOptRank];
#pragma unroll
            for (int cc = 0; cc < kOptRank; ++cc) nv[cc] = 0.0;
#pragma unroll
            for (int r = 0; r < kOptRank; ++r) {
                if (r < Rk) {
#pragma unroll
                    for (int cc = 0; cc < kOptRank; ++cc)
                        if (cc < Rk1) nv[cc] += v[r] * (double)A[r + Rk * cc];
                }
            }
#pragma unroll
            for (int cc = 0; cc < kOptRank; ++cc) v[cc] = nv[cc];
        }
#pragma unroll
        for (int r = 0; r < kOptRank; ++r)
            if (r < Rn) sS[c][r + Rn * s] = v[r];
    }
    // Wavefront w takes the block's columns 16 w .. 16 w + 15.  Its fiber
    // entries are requested before the barrier, in the layout of the matrix
    // core's result: lane l holds column 16 w + l % 16 at rows
    // 16 rt + 4 e + l / 16 (row tile rt, entry e of the 16 x 16 result).
    const int lane = tid & 63, wv = tid >> 6, lc = lane & 15, lk = lane >> 4;
    const int c = wv * 16 + lc;
    const int64_t jc = j0 + c;
    const bool colok = jc < J;
    const TX* Xn = static_cast<const TX*>(xs.rep[n]);
    const int RT = (In + 15) >> 4, KS = (RR + 3) >> 2;
    double xv[4 * Q][4];
#pragma unroll
    for (int rt = 0; rt < 4 * Q; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 16 * rt + 4 * e + lk;
            xv[rt][e] = (colok && i < In) ? to_f64(Xn[jc * In + i]) : 0.0;
        }
    __syncthreads();
    if (tid < kOptCols) {
        double ss = 0.0;
        for (int cc = 0; cc < RR; ++cc) ss += sS[tid][cc] * sS[tid][cc];
        sN[tid] = ss;
    }
    // pred = G_{n(2)} s_j on the FP64 matrix cores, K = 4 entries of s_j per
    // instruction: A[row][k] = G(16 rt + row, 4 ks + k) (lane l: row l % 16,
    // k = l / 16), B[k][col] = s_j(4 ks + k) of column 16 w + col (lane l:
    // k = l / 16, col = l % 16); entries past R_n R_{n+1} are zeros in sS.
    // (A operands loaded beside the fibers instead measured slower: the
    // extra registers cut the wavefronts per SIMD from 6 to 3.)
    typedef double od4 __attribute__((ext_vector_type(4)));
    const TC* Gn = static_cast<const TC*>(cores.p[n]);
    double bv[kOptRRMax / 4];
#pragma unroll
    for (int ks = 0; ks < kOptRRMax / 4; ++ks) bv[ks] = sS[c][4 * ks + lk];
    double rr = 0.0;
#pragma unroll
    for (int rt = 0; rt < 4 * Q; ++rt) {
        if (rt < RT) {
            od4 acc = {0.0, 0.0, 0.0, 0.0};
            const int gi = 16 * rt + lc;
#pragma unroll
            for (int ks = 0; ks < kOptRRMax / 4; ++ks) {
                if (ks < KS) {
                    const int gk = 4 * ks + lk;
                    const double av = (gi < In && gk < RR) ? (double)Gn[gi * RR + gk] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[ks], acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * rt + 4 * e + lk;
                const double r = xv[rt][e] - acc[e];
                rr += i < In ? r * r : 0.0;
            }
        }
    }
    // the four row groups of each column, in a fixed order
    rr += __shfl_xor(rr, 16, 64);
    rr += __shfl_xor(rr, 32, 64);
    __syncthreads();
    if (lk == 0 && colok) a[jc] = sqrt(rr) * sqrt(sN[c]);
}


// Per-block FP64 sums of a (fixed order within a block).
__global__ __launch_bounds__(kOptBlock) void k_opt_blocksum(tr_desc d, ModeSrc ms, const double* __restrict__ a,
                                                           double* __restrict__ bs) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    n = __builtin_amdgcn_readfirstlane(n);   // uniform: its table reads stay scalar
    const int64_t J = J_of(d, n);
    const int64_t nb = (J + kOptBlock - 1) / kOptBlock;
    if (blockIdx.x >= nb) return;
    const int64_t j = (int64_t)blockIdx.x * kOptBlock + threadIdx.x;
    __shared__ double red[kOptBlock / 64];
    const double s = block_sum(j < J ? a[j] : 0.0, red);
    if (threadIdx.x == 0) bs[blockIdx.x] = s;
}

// Total, quantisation and per-block weight sums; then the block offsets.
__global__ __launch_bounds__(kOptBlock) void k_opt_quantize(tr_desc d, ModeSrc ms, const double* __restrict__ a,
                                                           const double* __restrict__ bs, uint64_t* __restrict__ w,
                                                           uint64_t* __restrict__ wbs, int32_t* status) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    n = __builtin_amdgcn_readfirstlane(n);   // uniform: its table reads stay scalar
    const int64_t J = J_of(d, n);
    const int64_t nb = (J + kOptBlock - 1) / kOptBlock;
    if (blockIdx.x >= nb) return;
    // the total of the block sums, the same fixed order in every block
    double part = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kOptBlock) part += bs[b];
    __shared__ double red[kOptBlock / 64];
    const double tot = block_sum(part, red);
    const bool zero = !(tot > 0.0) || !isfinite(tot);
    if (zero && blockIdx.x == 0 && threadIdx.x == 0) set_status(status, TR_DEV_ZERO_DIST);
    const int64_t j = (int64_t)blockIdx.x * kOptBlock + threadIdx.x;
    uint64_t wv = 0;
    if (j < J) {
        wv = zero ? quantize(1.0 / (double)J) : quantize(a[j] / tot);
        w[j] = wv;
    }
    // Inclusive scan inside the block (Hillis-Steele over 256 entries).
    __shared__ uint64_t sc[kOptBlock];
    sc[threadIdx.x] = wv;
    __syncthreads();
    for (int o = 1; o < kOptBlock; o <<= 1) {
        const uint64_t v = (int)threadIdx.x >= o ? sc[threadIdx.x - o] : 0ull;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    if (j < J) w[j] = sc[threadIdx.x];
    if (threadIdx.x == kOptBlock - 1) wbs[blockIdx.x] = sc[threadIdx.x];
}

__global__ __launch_bounds__(1024) void k_opt_offsets(tr_desc d, ModeSrc ms, uint64_t* __restrict__ wbs) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    n = __builtin_amdgcn_readfirstlane(n);   // uniform: its table reads stay scalar
    const int64_t J = J_of(d, n);
    const int64_t nb = (J + kOptBlock - 1) / kOptBlock;
    // exclusive scan of the block totals, in place: the inclusive scan
    // (integer sums, exact), then every entry takes its predecessor's value,
    // each thread shifting its own segment (the one entry it reads from the
    // segment before is read ahead of a barrier)
    block_scan_u64(wbs, nb);
    const int T = blockDim.x;
    const int64_t per = (nb + T - 1) / T;
    const int64_t b = threadIdx.x * per, e = min(nb, b + per);
    const uint64_t prev = (b > 0 && b < nb) ? wbs[b - 1] : 0ull;
    __syncthreads();
    for (int64_t i = e - 1; i > b; --i) wbs[i] = wbs[i - 1];
    if (b < nb) wbs[b] = prev;
}

__global__ __launch_bounds__(kOptBlock) void k_opt_apply(tr_desc d, ModeSrc ms, const uint64_t* __restrict__ wbs,
                                                        uint64_t* __restrict__ w) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    n = __builtin_amdgcn_readfirstlane(n);   // uniform: its table reads stay scalar
    const int64_t J = J_of(d, n);
    const int64_t j = (int64_t)blockIdx.x * kOptBlock + threadIdx.x;
    if (j < J) w[j] += wbs[blockIdx.x];
}

size_t dist_opt_ws_bytes(const tr_desc& d) {
    const Shape sh = shape_of(d);
    const int64_t nb = (sh.maxJ + kOptBlock - 1) / kOptBlock;
    return align_up((size_t)sh.maxJ * 8) + 2 * align_up((size_t)nb * 8);
}

hipError_t launch_dist_optimal(const tr_desc& d, ModeSrc ms, Ptrs cores, XSrc xs, uint64_t* cdf_J, int32_t* status,
                               void* ws, hipStream_t st) {
    const Shape sh = shape_of(d);
    const int64_t nb = (sh.maxJ + kOptBlock - 1) / kOptBlock;
    char* w = static_cast<char*>(ws);
    double* a = reinterpret_cast<double*>(w);
    double* bs = reinterpret_cast<double*>(w + align_up((size_t)sh.maxJ * 8));
    uint64_t* wbs = reinterpret_cast<uint64_t*>(w + align_up((size_t)sh.maxJ * 8) + align_up((size_t)nb * 8));
    const dim3 grid((unsigned)nb);
    const bool f64 = d.core_dtype == TR_F64;
    bool reps = true;
    for (int k = 0; k < d.N; ++k) reps = reps && xs.rep[k] != nullptr;
    if (reps && sh.maxI <= 128 && sh.maxRR <= kOptRRMax && sh.maxR <= kOptRank &&
        sh.maxJ < ((int64_t)1 << 31)) {
        const dim3 gr((unsigned)((sh.maxJ + kOptCols - 1) / kOptCols));
        const bool one = sh.maxI <= 64;
        if (f64 && d.x_dtype == TR_F64) {
            if (one) hipLaunchKernelGGL((k_opt_terms_rep<double, double, 1>), gr, dim3(256), 0, st, d, ms, cores, xs, a);
            else hipLaunchKernelGGL((k_opt_terms_rep<double, double, 2>), gr, dim3(256), 0, st, d, ms, cores, xs, a);
        } else if (!f64 && d.x_dtype == TR_F32) {
            if (one) hipLaunchKernelGGL((k_opt_terms_rep<float, float, 1>), gr, dim3(256), 0, st, d, ms, cores, xs, a);
            else hipLaunchKernelGGL((k_opt_terms_rep<float, float, 2>), gr, dim3(256), 0, st, d, ms, cores, xs, a);
        } else if (!f64 && d.x_dtype == TR_F16) {
            if (one) hipLaunchKernelGGL((k_opt_terms_rep<float, __half, 1>), gr, dim3(256), 0, st, d, ms, cores, xs, a);
            else hipLaunchKernelGGL((k_opt_terms_rep<float, __half, 2>), gr, dim3(256), 0, st, d, ms, cores, xs, a);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (f64 && d.x_dtype == TR_F64)
        hipLaunchKernelGGL((k_opt_terms<double, double>), grid, dim3(kOptBlock), 0, st, d, ms, cores, xs, a);
    else if (!f64 && d.x_dtype == TR_F32)
        hipLaunchKernelGGL((k_opt_terms<float, float>), grid, dim3(kOptBlock), 0, st, d, ms, cores, xs, a);
    else if (!f64 && d.x_dtype == TR_F16)
        hipLaunchKernelGGL((k_opt_terms<float, __half>), grid, dim3(kOptBlock), 0, st, d, ms, cores, xs, a);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_opt_blocksum, grid, dim3(kOptBlock), 0, st, d, ms, a, bs);
    hipLaunchKernelGGL(k_opt_quantize, grid, dim3(kOptBlock), 0, st, d, ms, a, bs, cdf_J, wbs, status);
    hipLaunchKernelGGL(k_opt_offsets, dim3(1), dim3(1024), 0, st, d, ms, wbs);
    hipLaunchKernelGGL(k_opt_apply, grid, dim3(kOptBlock), 0, st, d, ms, wbs, cdf_J);
    return hipGetLastError();
}

}  // namespace trk
