// a1/a3/a4: mode pick, index draws with their probabilities, and the sampled
// rows of the subchain matrix (Algorithm SSDTP).
//
// One thread per (sample f, row s of M_f).  Every thread of a sample draws
// the sample's indices itself (a few Philox blocks: cheaper than a barrier),
// the s == 0 thread stores idx and p_F.  The row s of
// M_f = G_{n+1}(i_{n+1}) ... G_{n-1}(i_{n-1}) starts as e_s and is carried
// through the chain in registers: v <- v * G_k(i_k), R_k x R_{k+1} slices
// read from L1/L2 (cores are small).  The thread writes S[f][r + R_n s] for
// r < R_n: the R_{n+1} threads of a sample write one contiguous row.
#include "internal.hpp"

namespace trk {

template <typename TC>
__global__ __launch_bounds__(256) void k_sample_subchain(tr_desc d, ModeSrc ms, int m, CdfPtrs cdf,
                                                         const uint64_t* __restrict__ cdf_J,
                                                         int stream_tag, Ptrs cores,
                                                         int32_t* __restrict__ idx,
                                                         double* __restrict__ pF,
                                                         TC* __restrict__ S, int do_sample,
                                                         int do_subchain) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int N = d.N;
    const int n1 = ring_next(n, N);
    const int Rn = d.R[n], Rn1 = d.R[n1];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t f = gid / Rn1;
    const int s = (int)(gid - f * Rn1);
    if (f >= m) return;

    int ik[kMaxOrder];
    if (do_sample) {
        double p = 1.0;
        if (cdf_J) {
            const int64_t J = J_of(d, n);
            const uint64_t r = draw_word(ms.seed, t, (uint64_t)f, (uint64_t)n, (uint64_t)stream_tag);
            double pj;
            int64_t j;
            {   // first j with cdf_J[j] > u over [0, J)
                const uint64_t W = cdf_J[J - 1];
                const uint64_t u = mulhi64(r, W);
                int64_t lo = 0, hi = J - 1;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (cdf_J[mid] > u) hi = mid; else lo = mid + 1;
                }
                const uint64_t prev = lo > 0 ? cdf_J[lo - 1] : 0ull;
                pj = (double)(cdf_J[lo] - prev) / (double)W;
                j = lo;
            }
            p = pj;
            int k = n1;
            for (int q = 1; q < N; ++q) {
                ik[k] = (int)(j % d.I[k]);
                j /= d.I[k];
                k = ring_next(k, N);
            }
        } else {
            int k = n1;
            for (int q = 1; q < N; ++q) {
                const uint64_t r = draw_word(ms.seed, t, (uint64_t)f, (uint64_t)k, (uint64_t)stream_tag);
                double pk;
                if (cdf.p[k]) {
                    ik[k] = cdf_pick(cdf.p[k], d.I[k], r, &pk);
                } else {
                    ik[k] = (int)mulhi64(r, (uint64_t)d.I[k]);
                    pk = 1.0 / (double)d.I[k];
                }
                p = p * pk;
                k = ring_next(k, N);
            }
        }
        ik[n] = -1;
        if (s == 0) {
            for (int k = 0; k < N; ++k) idx[f * N + k] = ik[k];
            pF[f] = p;
        }
    } else {
        bool ok = true;
        for (int k = 0; k < N; ++k) {
            ik[k] = idx[f * N + k];
            if (k != n && (ik[k] < 0 || ik[k] >= d.I[k])) ok = false;
        }
        if (!ok) {   // invalid caller index: the row is NaN, nothing is read
            TC* out = S + f * (int64_t)(Rn * Rn1) + (int64_t)Rn * s;
            for (int r = 0; r < Rn; ++r) out[r] = TC(NAN);
            return;
        }
    }
    if (!do_subchain) return;

    // Row s of M_f through the chain n+1, ..., n-1.
    TC v[kMaxRank];
    int k = n1;
    {
        const TC* A = static_cast<const TC*>(cores.p[k]) + (int64_t)ik[k] * d.R[k] * d.R[ring_next(k, N)];
        const int Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
#pragma unroll
        for (int c = 0; c < kMaxRank; ++c) v[c] = c < Rk1 ? A[s + Rk * c] : TC(0);
    }
    for (int q = 2; q < N; ++q) {
        k = ring_next(k, N);
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
    TC* out = S + f * (int64_t)(Rn * Rn1) + (int64_t)Rn * s;
#pragma unroll
    for (int r = 0; r < kMaxRank; ++r)
        if (r < Rn) out[r] = v[r];
}

hipError_t launch_sample_subchain(const tr_desc& d, ModeSrc ms, int m, CdfPtrs cdf,
                                  const uint64_t* cdf_J, int stream_tag, Ptrs cores,
                                  int32_t* idx, double* pF, void* S, bool do_sample,
                                  bool do_subchain, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const Shape sh = shape_of(d);
    const int64_t threads = (int64_t)m * sh.maxR;
    const dim3 grid((unsigned)((threads + 255) / 256));
    if (d.core_dtype == TR_F64)
        hipLaunchKernelGGL(k_sample_subchain<double>, grid, dim3(256), 0, st, d, ms, m, cdf, cdf_J,
                           stream_tag, cores, idx, pF, static_cast<double*>(S), (int)do_sample,
                           (int)do_subchain);
    else
        hipLaunchKernelGGL(k_sample_subchain<float>, grid, dim3(256), 0, st, d, ms, m, cdf, cdf_J,
                           stream_tag, cores, idx, pF, static_cast<float*>(S), (int)do_sample,
                           (int)do_subchain);
    return hipGetLastError();
}

}  // namespace trk
