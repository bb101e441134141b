// a2: the sampling laws of Section 3.2 turned into integer-weight CDFs.
//
//   Euclidean (Lemma euc_est): p(i) = ||G_k(:,i,:)||_F^2 / ||G_k||_F^2.
//   Leverage (Lemma lev_est):  p(i) = l_i(G_{k(2)}) / rank, l_i = ||L^{-1} g_i||^2
//                              with L L^T the FP64 Gram G_{k(2)}^T G_{k(2)}.
//   Optimal (eq:optimal_prob): q(j) ~ ||X_[n](:,j) - G_{n(2)} s_j|| * ||s_j||
//                              over the J_n columns, FP64.
// Weights w = floor(p 2^40) + 1 and their inclusive prefix sums are exact
// integers: the sampler's choice depends only on them.
#include "internal.hpp"

namespace trk {

constexpr double kTwo40 = 1099511627776.0;

// Inclusive scan of a[0..len) (uint64) by one block, in place.
__device__ inline void block_scan_u64(uint64_t* a, int64_t len) {
    __shared__ uint64_t part[1024];
    const int T = blockDim.x;
    const int64_t per = (len + T - 1) / T;
    const int64_t b = threadIdx.x * per, e = min(len, b + per);
    uint64_t s = 0;
    for (int64_t i = b; i < e; ++i) {
        s += a[i];
        a[i] = s;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int i = 0; i < T; ++i) {
            const uint64_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    const uint64_t off = part[threadIdx.x];
    for (int64_t i = b; i < e; ++i) a[i] += off;
    __syncthreads();
}

__device__ inline uint64_t quantize(double p) { return (uint64_t)floor(p * kTwo40) + 1ull; }

__device__ inline void write_uniform_weights(uint64_t* w, int64_t len) {
    const uint64_t wu = quantize(1.0 / (double)len);
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) w[i] = wu;
    __syncthreads();
}

// Euclidean law of core k (one block).
template <typename TC>
__global__ __launch_bounds__(1024) void k_dist_euclid(tr_desc d, ModeSrc ms, int use_mode, int k_fixed,
                                                      Ptrs cores, MutPtrs cdf_out, int32_t* status) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    const int RR = d.R[k] * d.R[ring_next(k, d.N)];
    const TC* G = static_cast<const TC*>(cores.p[k]);
    uint64_t* w = static_cast<uint64_t*>(cdf_out.p[k]);
    double* rn = reinterpret_cast<double*>(w);   // row norms staged in the output
    double loc = 0.0;   // this thread's rows, then a fixed-order block sum
    for (int i = threadIdx.x; i < Ik; i += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < RR; ++c) {
            const double v = (double)G[(int64_t)i * RR + c];
            s += v * v;
        }
        rn[i] = s;
        loc += s;
    }
    __shared__ double red[16];
    const double tot = block_sum(loc, red);
    if (!(tot > 0.0) || !isfinite(tot)) {
        if (threadIdx.x == 0) set_status(status, TR_DEV_ZERO_DIST);
        write_uniform_weights(w, Ik);
    } else {
        for (int i = threadIdx.x; i < Ik; i += blockDim.x) w[i] = quantize(rn[i] / tot);
        __syncthreads();
    }
    block_scan_u64(w, Ik);
}

// Leverage law of core k (one block): Gram, Cholesky, row solves.
template <typename TC>
__global__ __launch_bounds__(1024) void k_dist_leverage(tr_desc d, ModeSrc ms, int use_mode, int k_fixed,
                                                        Ptrs cores, MutPtrs cdf_out, int32_t* status,
                                                        double* __restrict__ A) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    const int RR = d.R[k] * d.R[ring_next(k, d.N)];
    const TC* G = static_cast<const TC*>(cores.p[k]);
    uint64_t* w = static_cast<uint64_t*>(cdf_out.p[k]);
    double* lev = reinterpret_cast<double*>(w);
    if (Ik <= RR) {   // full row rank taken: every leverage score is 1
        write_uniform_weights(w, Ik);
        block_scan_u64(w, Ik);
        return;
    }
    for (int e = threadIdx.x; e < RR * RR; e += blockDim.x) {
        const int a = e % RR, b = e / RR;
        double s = 0.0;
        for (int i = 0; i < Ik; ++i) s += (double)G[(int64_t)i * RR + a] * (double)G[(int64_t)i * RR + b];
        A[e] = s;
    }
    __syncthreads();
    // Right-looking Cholesky in A (column-major).
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    for (int j = 0; j < RR; ++j) {
        __syncthreads();
        const double djj = A[j + (int64_t)RR * j];
        if (!(djj > 0.0) || !isfinite(djj)) {
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
    if (bad) {
        if (threadIdx.x == 0) set_status(status, TR_DEV_NOT_SPD);
        write_uniform_weights(w, Ik);
        block_scan_u64(w, Ik);
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
    block_scan_u64(w, Ik);
}

// The same law for R_k R_{k+1} <= 128 with the factor kept in LDS (one
// block of 1024 threads): (1) the lower triangle of A = G^T G, rows of G
// staged through LDS in chunks, every entry summed over i ascending; (2)
// right-looking Cholesky A = L L^T; (3) L^{-1} in place, column by column
// from the last (column j below the diagonal is -(1/L_jj) L22^{-1} L(j+1:, j)
// with L22^{-1} already formed); (4) l_i = ||L^{-1} g_i||^2, the rows of G
// staged again, each row's RR entries of L^{-1} g_i split over a group of
// threads and their squares summed by a shuffle reduction.
constexpr int kLevThreads = 1024;

static int lev_chunk_rows(int RR, int es) {
    // the block scan's 8 KiB and a few words of static LDS come on top
    const int budget = 160 * 1024 - 8192 - 1024 - RR * RR * 8 - RR * 8;
    int cr = budget / (RR * es);
    cr = cr > 64 ? 64 : cr;
    return cr < 1 ? 1 : cr;
}

template <typename TC>
__global__ __launch_bounds__(kLevThreads) void k_dist_leverage_lds(tr_desc d, ModeSrc ms, int use_mode, int k_fixed,
                                                                  Ptrs cores, MutPtrs cdf_out, int32_t* status,
                                                                  int CR) {
    uint64_t t;
    int k = k_fixed;
    if (use_mode) resolve_mode(ms, d.N, &t, &k);
    const int Ik = d.I[k];
    const int RR = d.R[k] * d.R[ring_next(k, d.N)];
    const TC* G = static_cast<const TC*>(cores.p[k]);
    uint64_t* w = static_cast<uint64_t*>(cdf_out.p[k]);
    double* lev = reinterpret_cast<double*>(w);
    const int tid = threadIdx.x;
    if (Ik <= RR) {   // full row rank taken: every leverage score is 1
        write_uniform_weights(w, Ik);
        block_scan_u64(w, Ik);
        return;
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sA = reinterpret_cast<double*>(smem_raw);   // RR x RR, column-major, lower triangle
    double* scol = sA + RR * RR;                         // [RR]
    TC* sG = reinterpret_cast<TC*>(scol + RR);          // [CR][RR], rows of G in the core dtype
    __shared__ int bad;

    // (1) Gram, lower triangle; entry q of the column-major lower triangle is
    // (a, b), a >= b, accumulated in place over the chunks of rows
    const int ntri = RR * (RR + 1) / 2;
    auto tri = [&](int q, int& ra, int& cb) {
        // column: the largest c with c RR - c (c - 1) / 2 <= q
        const double t2 = 2.0 * RR + 1.0;
        int c = (int)((t2 - sqrt(t2 * t2 - 8.0 * q)) * 0.5);
        c = c < 0 ? 0 : (c >= RR ? RR - 1 : c);
        while (c > 0 && c * RR - c * (c - 1) / 2 > q) --c;
        while (c + 1 < RR && (c + 1) * RR - (c + 1) * c / 2 <= q) ++c;
        cb = c;
        ra = c + (q - (c * RR - c * (c - 1) / 2));
    };
    for (int q = tid; q < ntri; q += kLevThreads) {
        int ra, cb;
        tri(q, ra, cb);
        sA[ra + RR * cb] = 0.0;
    }
    for (int r0 = 0; r0 < Ik; r0 += CR) {
        const int nr = min(CR, Ik - r0);
        __syncthreads();
        for (int e = tid; e < nr * RR; e += kLevThreads) sG[e] = G[(int64_t)r0 * RR + e];
        __syncthreads();
        for (int q = tid; q < ntri; q += kLevThreads) {
            int ra, cb;
            tri(q, ra, cb);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;   // four chains hide the LDS latency
            int r = 0;
            for (; r + 3 < nr; r += 4) {
                s0 += (double)sG[r * RR + ra] * (double)sG[r * RR + cb];
                s1 += (double)sG[(r + 1) * RR + ra] * (double)sG[(r + 1) * RR + cb];
                s2 += (double)sG[(r + 2) * RR + ra] * (double)sG[(r + 2) * RR + cb];
                s3 += (double)sG[(r + 3) * RR + ra] * (double)sG[(r + 3) * RR + cb];
            }
            for (; r < nr; ++r) s0 += (double)sG[r * RR + ra] * (double)sG[r * RR + cb];
            sA[ra + RR * cb] += (s0 + s1) + (s2 + s3);
        }
    }
    if (tid == 0) bad = 0;
    // (2) Cholesky
    for (int j = 0; j < RR; ++j) {
        __syncthreads();
        const double djj = sA[j + RR * j];
        if (!(djj > 0.0) || !isfinite(djj)) {
            if (tid == 0) bad = 1;
            break;
        }
        const double ljj = sqrt(djj);
        __syncthreads();
        for (int i = j + tid; i < RR; i += kLevThreads) sA[i + RR * j] = i == j ? ljj : sA[i + RR * j] / ljj;
        __syncthreads();
        const int wd = RR - j - 1;
        for (int e = tid; e < wd * wd; e += kLevThreads) {
            const int i = j + 1 + e % wd, c = j + 1 + e / wd;
            if (c <= i) sA[i + RR * c] -= sA[i + RR * j] * sA[c + RR * j];
        }
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) set_status(status, TR_DEV_NOT_SPD);
        write_uniform_weights(w, Ik);
        block_scan_u64(w, Ik);
        return;
    }
    // (3) L^{-1} in place
    for (int j = RR - 1; j >= 0; --j) {
        for (int i = j + 1 + tid; i < RR; i += kLevThreads) scol[i] = sA[i + RR * j];
        __syncthreads();
        const double dj = 1.0 / sA[j + RR * j];
        double x = 0.0;
        const int i = j + 1 + tid;
        if (i < RR) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int c = j + 1;
            for (; c + 3 <= i; c += 4) {
                s0 += sA[i + RR * c] * scol[c];
                s1 += sA[i + RR * (c + 1)] * scol[c + 1];
                s2 += sA[i + RR * (c + 2)] * scol[c + 2];
                s3 += sA[i + RR * (c + 3)] * scol[c + 3];
            }
            for (; c <= i; ++c) s0 += sA[i + RR * c] * scol[c];
            x = -dj * ((s0 + s1) + (s2 + s3));
        }
        __syncthreads();
        if (i < RR) sA[i + RR * j] = x;
        if (tid == 0) sA[j + RR * j] = dj;
    }
    __syncthreads();
    // (4) leverage scores, TPR threads per row
    int TPR = 8;   // threads per row: rows per round = 1024 / TPR <= CR (CR >= 16 for RR <= 128)
    while (TPR < 64 && TPR * CR < kLevThreads) TPR <<= 1;
    const int RPB = kLevThreads / TPR;
    for (int r0 = 0; r0 < Ik; r0 += RPB) {
        const int nr = min(RPB, Ik - r0);
        __syncthreads();
        for (int e = tid; e < nr * RR; e += kLevThreads) sG[e] = G[(int64_t)r0 * RR + e];
        __syncthreads();
        const int rl = tid / TPR, sub = tid - rl * TPR;
        double s2 = 0.0;
        if (rl < nr) {
            const TC* g = sG + rl * RR;
            for (int j = sub; j < RR; j += TPR) {
                double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
                int c = 0;
                for (; c + 3 <= j; c += 4) {
                    v0 += sA[j + RR * c] * (double)g[c];
                    v1 += sA[j + RR * (c + 1)] * (double)g[c + 1];
                    v2 += sA[j + RR * (c + 2)] * (double)g[c + 2];
                    v3 += sA[j + RR * (c + 3)] * (double)g[c + 3];
                }
                for (; c <= j; ++c) v0 += sA[j + RR * c] * (double)g[c];
                const double v = (v0 + v1) + (v2 + v3);
                s2 += v * v;
            }
        }
        for (int o = TPR >> 1; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
        if (rl < nr && sub == 0) lev[r0 + rl] = s2;
    }
    __syncthreads();
    for (int i = tid; i < Ik; i += kLevThreads) w[i] = quantize(lev[i] / (double)RR);
    __syncthreads();
    block_scan_u64(w, Ik);
}

size_t dist_ws_bytes(const tr_desc& d, int law) {
    const Shape sh = shape_of(d);
    return law == TR_LAW_LEVERAGE ? align_up((size_t)sh.maxRR * sh.maxRR * 8) : 256;
}

hipError_t launch_dist(const tr_desc& d, ModeSrc ms, bool use_mode, int k, int law, Ptrs cores,
                       uint64_t* const* cdf_out, int32_t* status, void* ws, hipStream_t st) {
    MutPtrs out{};
    for (int q = 0; q < d.N; ++q) out.p[q] = cdf_out[q];
    const bool f64 = d.core_dtype == TR_F64;
    if (law == TR_LAW_EUCLID) {
        if (f64)
            hipLaunchKernelGGL(k_dist_euclid<double>, dim3(1), dim3(1024), 0, st, d, ms, (int)use_mode, k, cores,
                               out, status);
        else
            hipLaunchKernelGGL(k_dist_euclid<float>, dim3(1), dim3(1024), 0, st, d, ms, (int)use_mode, k, cores,
                               out, status);
    } else if (law == TR_LAW_LEVERAGE && shape_of(d).maxRR <= 128) {
        const int RR = use_mode ? shape_of(d).maxRR : d.R[k] * d.R[(k + 1) % d.N];
        const int es = f64 ? 8 : 4;
        const int CR = lev_chunk_rows(RR, es);
        const size_t shm = (size_t)RR * RR * 8 + (size_t)RR * 8 + (size_t)CR * RR * es;
#define TRK_LEV(TC)                                                                                         \
    do {                                                                                                    \
        if (!allow_lds(reinterpret_cast<const void*>(&k_dist_leverage_lds<TC>), shm)) return hipErrorInvalidValue; \
        hipLaunchKernelGGL(k_dist_leverage_lds<TC>, dim3(1), dim3(kLevThreads), shm, st, d, ms, (int)use_mode, k,  \
                           cores, out, status, CR);                                                         \
    } while (0)
        if (f64) TRK_LEV(double);
        else TRK_LEV(float);
#undef TRK_LEV
    } else if (law == TR_LAW_LEVERAGE) {
        double* A = static_cast<double*>(ws);
        if (f64)
            hipLaunchKernelGGL(k_dist_leverage<double>, dim3(1), dim3(1024), 0, st, d, ms, (int)use_mode, k,
                               cores, out, status, A);
        else
            hipLaunchKernelGGL(k_dist_leverage<float>, dim3(1), dim3(1024), 0, st, d, ms, (int)use_mode, k,
                               cores, out, status, A);
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

// Per-block FP64 sums of a (fixed order within a block).
__global__ __launch_bounds__(kOptBlock) void k_opt_blocksum(tr_desc d, ModeSrc ms, const double* __restrict__ a,
                                                           double* __restrict__ bs) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
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
    const int64_t J = J_of(d, n);
    const int64_t nb = (J + kOptBlock - 1) / kOptBlock;
    if (blockIdx.x >= nb) return;
    __shared__ double tot_s;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int64_t b = 0; b < nb; ++b) s += bs[b];
        tot_s = s;
    }
    __syncthreads();
    const double tot = tot_s;
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
        const uint64_t v = threadIdx.x >= o ? sc[threadIdx.x - o] : 0ull;
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
    const int64_t J = J_of(d, n);
    const int64_t nb = (J + kOptBlock - 1) / kOptBlock;
    // exclusive scan of the block totals, in place
    __shared__ uint64_t part[1024];
    const int T = blockDim.x;
    const int64_t per = (nb + T - 1) / T;
    const int64_t b = threadIdx.x * per, e = min(nb, b + per);
    uint64_t s = 0;
    for (int64_t i = b; i < e; ++i) {
        const uint64_t v = wbs[i];
        wbs[i] = s;
        s += v;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int i = 0; i < T; ++i) {
            const uint64_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    for (int64_t i = b; i < e; ++i) wbs[i] += part[threadIdx.x];
}

__global__ __launch_bounds__(kOptBlock) void k_opt_apply(tr_desc d, ModeSrc ms, const uint64_t* __restrict__ wbs,
                                                        uint64_t* __restrict__ w) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
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
    if (f64 && d.x_dtype == TR_F64)
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
