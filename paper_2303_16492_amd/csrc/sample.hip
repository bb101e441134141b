// a1/a3/a4: mode pick, index draws with their probabilities, and the sampled
// rows of the subchain matrix (Algorithm SSDTP).
//
// S[f][r + R_n s] = M_f(s, r) with M_f = G_{n+1}(i_{n+1}) ... G_{n-1}(i_{n-1})
// (the product of slices of the subchain, Section 3.2).
#include "internal.hpp"

namespace trk {

// A block takes SB samples.  Phase 1: one thread per (sample, mode) draws
// the index (the optimal law: one thread per sample draws over J_n); the
// probabilities are multiplied per sample in the order n+1, ..., n-1.  When
// the kernel draws the step's mode itself and the law is one per mode, the
// index draws do not depend on the mode: threads draw for every mode of
// every sample and one more thread draws the mode, all in the same Philox
// instruction stream, instead of one chain after the other; a draw for the
// step's own mode is dropped.
// do_sample == 2 enumerates instead: sample f is column j = f of X_[n]
// (every column once, m = J_n), decoded in the cyclic order, p = 1/J_n.
// Phase 2: the N-1 core slices of every sample are copied to LDS in one
// batch (a slice G_k(i) is row i of G_k(2): R_k R_{k+1} contiguous values).
// Phase 3: the chain products M <- M G_k(i_k), the last product written
// straight to S[f][r + R_n s] = M_f(s, r): for FP32 cores one wavefront per
// sample on the matrix cores; for FP64 one output entry per thread at a time
// (consecutive threads, consecutive columns), accumulated in FP64 with the
// inner index ascending.
template <typename TC>
__global__ __launch_bounds__(256) void k_sample_subchain(tr_desc d, ModeSrc ms, int m, int SB, CdfPtrs cdf,
                                                         const uint64_t* __restrict__ cdf_J, int stream_tag,
                                                         Ptrs cores, int32_t* __restrict__ idx, double* __restrict__ pF,
                                                         TC* __restrict__ S, int do_sample, int do_subchain) {
    const int N = d.N, tid = threadIdx.x;
    const int f0 = blockIdx.x * SB;
    const int nb = min(SB, m - f0);
    uint64_t t;
    int n;
    // per-mode laws with the mode drawn here: the draws of every mode beside
    // the mode's draw (thread nb N), one Philox chain per thread
    const bool early_draws = do_sample == 1 && !cdf_J && ms.n == -1;
    static_assert(16 * kMaxOrder + 1 <= 256, "one thread per (sample, mode) and one for the mode");
    int dr_i = 0;
    double dr_p = 0.0;
    if (early_draws) {
        __shared__ int s_mode;
        t = ms.t_dev ? *ms.t_dev : ms.t;
        if (tid <= nb * N) {
            const bool is_mode = tid == nb * N;
            const int fl = tid / N, k = tid - fl * N;
            const uint64_t r = draw_word(ms.seed, t, is_mode ? 0 : (uint64_t)(f0 + fl), is_mode ? 0 : (uint64_t)k,
                                         is_mode ? (uint64_t)TR_STREAM_MODE : (uint64_t)stream_tag);
            if (is_mode) {
                s_mode = (int)mulhi64(r, (uint64_t)N);
            } else {
                const gptr<uint64_t> ck = lane_pick_global<uint64_t>(cdf.p, k);   // k differs across lanes
                const int Ik = lane_pick(d.I, k);
                if (ck) {
                    dr_i = cdf_pick(ck, Ik, r, &dr_p);
                } else {
                    dr_i = (int)mulhi64(r, (uint64_t)Ik);
                    dr_p = 1.0 / (double)Ik;
                }
            }
        }
        __syncthreads();
        n = __builtin_amdgcn_readfirstlane(s_mode);   // uniform: what follows from it stays scalar
    } else {
        resolve_mode(ms, d.N, &t, &n);
    }
    if (ms.n_pub && blockIdx.x == 0 && threadIdx.x == 0) *ms.n_pub = n;
    const int n1 = ring_next(n, N);
    const int Rn = d.R[n], Rn1 = d.R[n1], RR = Rn * Rn1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int* sidx = reinterpret_cast<int*>(smem_raw);                   // [SB][kMaxOrder]
    double* sp = reinterpret_cast<double*>(sidx + SB * kMaxOrder);  // [SB][kMaxOrder], order of the chain
    int* sok = reinterpret_cast<int*>(sp + SB * kMaxOrder);         // [SB]
    TC* sl = reinterpret_cast<TC*>(sok + ((SB + 3) & ~3));          // slices, then two product buffers

    // chain order n+1, ..., n-1: stage q is mode (n + 1 + q) mod N; its
    // slice starts at soff[q] within a sample's slices
    __shared__ int soff[kMaxOrder + 1];
    if (tid == 0) {
        int o = 0;
        for (int q = 0; q < N - 1; ++q) {
            soff[q] = o;
            const int k = (n + 1 + q) % N;
            o += d.R[k] * d.R[ring_next(k, N)];
        }
        soff[N - 1] = o;
    }
    int mr = 0;   // largest rank: stride of the product buffers
    for (int k = 0; k < N; ++k) mr = max(mr, d.R[k]);
    if (do_sample == 2) {
        const int64_t J = J_of(d, n);
        for (int fl = tid; fl < nb; fl += blockDim.x) {
            int64_t j = f0 + fl;
            sp[fl * kMaxOrder] = 1.0 / (double)J;
            for (int q = 0; q < N - 1; ++q) {
                const int k = (n + 1 + q) % N;
                sidx[fl * kMaxOrder + k] = (int)(j % d.I[k]);
                j /= d.I[k];
            }
            sidx[fl * kMaxOrder + n] = -1;
            sok[fl] = 1;
        }
        __syncthreads();
    } else if (do_sample) {
        if (cdf_J) {
            for (int fl = tid; fl < nb; fl += blockDim.x) {
                const int64_t f = f0 + fl;
                const int64_t J = J_of(d, n);
                const uint64_t r = draw_word(ms.seed, t, (uint64_t)f, (uint64_t)n, (uint64_t)stream_tag);
                const uint64_t W = cdf_J[J - 1];
                const uint64_t u = mulhi64(r, W);
                int64_t lo = 0, hi = J - 1;   // first j with cdf_J[j] > u
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (cdf_J[mid] > u) hi = mid; else lo = mid + 1;
                }
                const uint64_t prev = lo > 0 ? cdf_J[lo - 1] : 0ull;
                sp[fl * kMaxOrder] = (double)(cdf_J[lo] - prev) / (double)W;
                int64_t j = lo;
                for (int q = 0; q < N - 1; ++q) {
                    const int k = (n + 1 + q) % N;
                    sidx[fl * kMaxOrder + k] = (int)(j % d.I[k]);
                    j /= d.I[k];
                }
                sidx[fl * kMaxOrder + n] = -1;
                sok[fl] = 1;
            }
        } else if (early_draws) {
            // thread (sample fl, mode k): its draw at chain position q
            if (tid < nb * N) {
                const int fl = tid / N, k = tid - fl * N;
                if (k == n) {
                    sidx[fl * kMaxOrder + n] = -1;
                    sok[fl] = 1;
                } else {
                    sidx[fl * kMaxOrder + k] = dr_i;
                    const int q = k - n - 1;   // position in the chain n+1, ..., n-1
                    sp[fl * kMaxOrder + (q < 0 ? q + N : q)] = dr_p;
                }
            }
        } else {
            for (int w = tid; w < nb * (N - 1); w += blockDim.x) {
                const int fl = w / (N - 1), q = w - fl * (N - 1);
                const int k = (n + 1 + q) % N;
                const uint64_t r = draw_word(ms.seed, t, (uint64_t)(f0 + fl), (uint64_t)k, (uint64_t)stream_tag);
                const gptr<uint64_t> ck = lane_pick_global<uint64_t>(cdf.p, k);   // k differs across lanes
                const int Ik = lane_pick(d.I, k);
                double pk;
                int i;
                if (ck) {
                    i = cdf_pick(ck, Ik, r, &pk);
                } else {
                    i = (int)mulhi64(r, (uint64_t)Ik);
                    pk = 1.0 / (double)Ik;
                }
                sidx[fl * kMaxOrder + k] = i;
                sp[fl * kMaxOrder + q] = pk;
                if (q == 0) {
                    sidx[fl * kMaxOrder + n] = -1;
                    sok[fl] = 1;
                }
            }
        }
        __syncthreads();
    } else {
        for (int fl = tid; fl < nb; fl += blockDim.x) {
            const int64_t f = f0 + fl;
            int ok = 1;
            for (int k = 0; k < N; ++k) {
                const int i = idx[f * N + k];
                sidx[fl * kMaxOrder + k] = i;
                if (k != n && (i < 0 || i >= d.I[k])) ok = 0;
            }
            sok[fl] = ok;   // invalid caller index: the row is NaN, nothing is read
        }
        __syncthreads();
    }
    // The draws and their probabilities go out after the slice loads are in
    // flight: a store issued before them would hold up their first wait.
    auto write_draws = [&]() {
        for (int fl = tid; fl < nb; fl += blockDim.x) {
            const int64_t f = f0 + fl;
            double p;
            if (cdf_J || do_sample == 2) {
                p = sp[fl * kMaxOrder];
            } else {
                p = 1.0;
                for (int q = 0; q < N - 1; ++q) p = p * sp[fl * kMaxOrder + q];
            }
            pF[f] = p;
            for (int k = 0; k < N; ++k) idx[f * N + k] = sidx[fl * kMaxOrder + k];
        }
    };
    if (!do_subchain) {
        if (do_sample) write_draws();
        return;
    }

    // Phase 2: slices of every sample, all loads in flight together.  Thread
    // w of a pass owns value w of every sample's slices (its slice q, mode k
    // and offset are the same for all samples), so the loads of the pass
    // are one per sample at a row taken from LDS: the row is clamped to 0
    // for a rejected caller index and the value masked afterwards, so no
    // load sits behind a branch.
    const int per = soff[N - 1];   // slice values per sample
    for (int w0 = 0; w0 < per; w0 += 256) {
        const int w = w0 + tid, wc = w < per ? w : per - 1;
        int q = 0;
        while (q + 1 < N - 1 && wc >= soff[q + 1]) ++q;
        const int k = (n + 1 + q) % N;
        const int len = soff[q + 1] - soff[q], off = wc - soff[q];
        const gptr<TC> src = lane_pick_global<TC>(cores.p, k);   // k differs across lanes
        constexpr int kSB = 16;   // samples per block at most
        int row[kSB];
        bool ok[kSB];
#pragma unroll
        for (int fl = 0; fl < kSB; ++fl) {   // sample indices clamped into the block's own
            const int fc = fl < nb ? fl : nb - 1;
            const int i = sidx[fc * kMaxOrder + k];
            ok[fl] = sok[fc] != 0;
            row[fl] = ok[fl] ? i : 0;
        }
        TC v[kSB];
#pragma unroll
        for (int fl = 0; fl < kSB; ++fl) v[fl] = src[(int64_t)row[fl] * len + off];
        if (w0 == 0 && do_sample) write_draws();   // while the loads above are in flight
#pragma unroll
        for (int fl = 0; fl < kSB; ++fl)
            if (fl < nb && w < per) sl[(size_t)fl * per + w] = ok[fl] ? v[fl] : TC(0);
    }
    __syncthreads();

    // Phase 3: M (R_{n+1} x R_{k+1}, row-major per sample, stride mr^2)
    // through the chain; slice q of sample fl holds (r, c) at
    // sl[fl * per + soff[q] + r + R_k c].  The last product goes to S.
    const size_t P2 = (size_t)mr * mr;
    TC* bufA = sl + (size_t)SB * per;
    TC* bufB = bufA + (size_t)SB * P2;
    if (N == 2) {
        for (int e = tid; e < nb * RR; e += blockDim.x) {
            const int fl = e / RR, w = e - fl * RR;
            const int s = w / Rn, r = w - s * Rn;
            S[(int64_t)(f0 + fl) * RR + w] = sok[fl] ? sl[(size_t)fl * per + s + Rn1 * r] : TC(NAN);
        }
        return;
    }
    if constexpr (sizeof(TC) == 4) {
        // FP32: one wavefront per sample (samples wv, wv + 4, ...): M <- M A_q
        // as a zero-padded 16 x 16 tile on the matrix cores (K = R_k in four
        // steps of 4); an intermediate M goes back through the wavefront's
        // LDS tile to become the next A operand.  Operand layouts of
        // v_mfma_f32_16x16x4_f32 (lane l): A[l % 16][l / 16], B[l / 16][l % 16],
        // D[4 (l / 16) + j][l % 16].
        typedef float sf4 __attribute__((ext_vector_type(4)));
        const int wv = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
        // product tiles after the slices (and after the FP64 path's product
        // buffers, which exist for N > 3 only)
        float* Mw = reinterpret_cast<float*>(bufA + (N > 3 ? 2 * (size_t)SB * P2 : 0)) + wv * 256;
        if (N == 3) {
            // One product per sample, M = A_0 A_1; the wavefront's samples
            // wv, wv + 4, wv + 8, wv + 12 (SB <= 16) side by side, operands
            // read at clamped indices and masked.
            const int k = (n + 2) % N, Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
            const int lrA = lr < Rn1 ? lr : Rn1 - 1, lrB = lr < Rk1 ? lr : Rk1 - 1;
            float a[4][4], b[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int fl = wv + 4 * u;
                const float* base = reinterpret_cast<const float*>(sl) + (size_t)(fl < nb ? fl : 0) * per;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int kk = 4 * ks + lk, kc = kk < Rk ? kk : Rk - 1;
                    // the masks multiply (a select would become a branch around
                    // each LDS read); a clamped entry is one of the sample's own
                    // and feeds the same outputs, so non-finite values propagate
                    // exactly as with zero padding
                    const float av = base[lrA + Rn1 * kc], bv = base[soff[1] + kc + Rk * lrB];
                    a[u][ks] = av * ((lr < Rn1 && kk < Rk) ? 1.f : 0.f);
                    b[u][ks] = bv * ((kk < Rk && lr < Rk1) ? 1.f : 0.f);
                }
            }
            sf4 acc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = sf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][ks], b[u][ks], acc[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int fl = wv + 4 * u;
                if (fl < nb) {   // uniform
                    const bool ok = sok[fl] != 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {   // S(f, r + R_n s) = M_f(s, r), s = 4 lk + j, r = lr
                        const int srow = 4 * lk + j;
                        if (srow < Rn1 && lr < Rn)
                            S[(int64_t)(f0 + fl) * RR + lr + Rn * srow] = ok ? (TC)acc[u][j] : TC(NAN);
                    }
                }
            }
            return;
        }
        for (int fl = wv; fl < nb; fl += (int)(blockDim.x >> 6)) {
            const float* base = reinterpret_cast<const float*>(sl) + (size_t)fl * per;
            sf4 mv = {0.f, 0.f, 0.f, 0.f};
            for (int q = 1; q < N - 1; ++q) {
                const int k = (n + 1 + q) % N, Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
                const float* Aq = base + soff[q];
                sf4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int kk = 4 * ks + lk;
                    float a;
                    if (q == 1) a = (lr < Rn1 && kk < Rk) ? base[lr + Rn1 * kk] : 0.f;   // first slice, row lr
                    else a = Mw[lr * 16 + kk];
                    const float b = (kk < Rk && lr < Rk1) ? Aq[kk + Rk * lr] : 0.f;
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
                }
                mv = acc;
                if (q + 1 < N - 1) {   // D rows 4 lk + j, column lr
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int j = 0; j < 4; ++j) Mw[(4 * lk + j) * 16 + lr] = mv[j];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_s_waitcnt(0xc07f);
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {   // S(f, r + R_n s) = M_f(s, r), s = 4 lk + j, r = lr
                const int srow = 4 * lk + j;
                if (srow < Rn1 && lr < Rn)
                    S[(int64_t)(f0 + fl) * RR + lr + Rn * srow] = sok[fl] ? (TC)mv[j] : TC(NAN);
            }
        }
        return;
    }
    const TC* Mc = nullptr;     // current product; null: the first slice
    int cols = d.R[ring_next(n1, N)];
    for (int q = 1; q < N - 1; ++q) {
        const int k = (n + 1 + q) % N, Rk = d.R[k], Rk1 = d.R[ring_next(k, N)];
        const bool last = q == N - 2;   // then Rk1 == R_n
        TC* Mo = (q & 1) ? bufA : bufB;
        for (int e = tid; e < nb * Rn1 * Rk1; e += blockDim.x) {
            const int fl = e / (Rn1 * Rk1), w = e - fl * (Rn1 * Rk1);
            const int s = w / Rk1, c = w - s * Rk1;
            const TC* A = sl + (size_t)fl * per + soff[q];
            TC acc = TC(0);
            for (int r = 0; r < Rk; ++r) {
                const TC mv = Mc ? Mc[(size_t)fl * P2 + s * cols + r] : sl[(size_t)fl * per + s + Rn1 * r];
                acc += mv * A[r + Rk * c];
            }
            if (last)
                S[(int64_t)(f0 + fl) * RR + w] = sok[fl] ? acc : TC(NAN);
            else
                Mo[(size_t)fl * P2 + s * Rk1 + c] = acc;
        }
        if (!last) __syncthreads();
        Mc = Mo;
        cols = Rk1;
    }
}

// Samples per block: the slices of all of them and two product buffers fit
// in 48 KiB of LDS.
static int sample_block(const tr_desc& d, const Shape& sh, size_t es, size_t* lds) {
    const size_t per = (size_t)(d.N - 1) * sh.maxR * sh.maxR;
    const size_t prod = d.N > 3 ? 2 * (size_t)sh.maxR * sh.maxR : 0;   // product buffers
    const size_t need = (per + prod) * es + kMaxOrder * 12 + 4;
    int SB = (int)((48 * 1024) / need);
    SB = SB < 1 ? 1 : (SB > 16 ? 16 : SB);   // the kernel's slice loads assume SB <= 16
    *lds = (size_t)SB * kMaxOrder * 12 + (size_t)((SB + 3) & ~3) * 4 + 16 +
           ((size_t)SB * per + (size_t)SB * prod) * es + (es == 4 ? 4 * 256 * 4 : 0);   // FP32: product tiles
    return SB;
}

hipError_t launch_sample_subchain(const tr_desc& d, ModeSrc ms, int m, CdfPtrs cdf,
                                  const uint64_t* cdf_J, int stream_tag, Ptrs cores,
                                  int32_t* idx, double* pF, void* S, bool do_sample,
                                  bool do_subchain, hipStream_t st) {
    return launch_sample_subchain_mode(d, ms, m, cdf, cdf_J, stream_tag, cores, idx, pF, S, do_sample ? 1 : 0,
                                       do_subchain, st);
}

hipError_t launch_sample_subchain_mode(const tr_desc& d, ModeSrc ms, int m, CdfPtrs cdf,
                                       const uint64_t* cdf_J, int stream_tag, Ptrs cores,
                                       int32_t* idx, double* pF, void* S, int sample_mode,
                                       bool do_subchain, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const Shape sh = shape_of(d);
    const size_t es = d.core_dtype == TR_F64 ? 8 : 4;
    size_t lds = 0;
    const int SB = sample_block(d, sh, es, &lds);
    const dim3 grid((unsigned)((m + SB - 1) / SB));
    if (d.core_dtype == TR_F64)
        hipLaunchKernelGGL(k_sample_subchain<double>, grid, dim3(256), lds, st, d, ms, m, SB, cdf, cdf_J,
                           stream_tag, cores, idx, pF, static_cast<double*>(S), sample_mode,
                           (int)do_subchain);
    else
        hipLaunchKernelGGL(k_sample_subchain<float>, grid, dim3(256), lds, st, d, ms, m, SB, cdf, cdf_J,
                           stream_tag, cores, idx, pF, static_cast<float*>(S), sample_mode,
                           (int)do_subchain);
    return hipGetLastError();
}

}  // namespace trk
