// a11: many independent TR problems (uneven order, sizes and ranks) advance
// by TR-BRSGD steps (Algorithm alg:TR_BRSGD with uniform fiber sampling) in
// one persistent launch: workgroup p owns problem p and runs all its steps
// itself, so problems never wait on each other and no grid-wide
// synchronisation exists.  One step of one problem:
//   mode n from (seed, t); per chunk of CH samples: Philox draws (one per
//   (sample, core)), the sampled subchain rows S (slice products, stored as
//   FP16 in LDS row-major and transposed), the fibers from the mode-major
//   replica, E = X_F - G_n S^T on FP16 matrix cores with FP32 accumulation
//   (E scaled by 1/(J_n p_f) and rounded to FP16), g += E S on FP16 matrix
//   cores into an FP32 LDS accumulator; then p = g / m (eq:S_gradient with
//   the sign of the direction folded in) and the step rule on the core.
// The loss estimate of the step is written in FP64.  The chunk size and the
// number of wavefronts are template parameters picked by the host tuner.
#include "internal.hpp"

namespace trk {

typedef float f32x4b __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int kBatchMaxI = 128;     // I_n
constexpr int kBatchMaxRR = 160;    // R_n R_{n+1} <= 144, padded to the K step (32)
constexpr int kBatchRank = 12;      // R_n
constexpr int kBatchGroup = 16;     // samples whose core slices are staged together
constexpr int kBatchMaxN = 5;       // order (slices per sample: N - 1)
// the FP32 slices of a group, each padded to 12 x 12
constexpr int kBatchSliceFloats = kBatchGroup * (kBatchMaxN - 1) * 12 * 12;

template <int CH>
struct BatchLds {
    static constexpr int SP = kBatchMaxRR + 8;   // pitch of S rows (FP16)
    static constexpr int TP = CH + 8;            // pitch of S^T and E rows (FP16)
    static constexpr size_t s_off = 0;
    static constexpr size_t t_off = s_off + (size_t)CH * SP * 2;
    static constexpr size_t e_off = t_off + (size_t)kBatchMaxRR * TP * 2;
    static constexpr size_t c_off = e_off + (size_t)kBatchMaxI * TP * 2;     // staged slices (FP32)
    static constexpr size_t m_off = c_off + (size_t)kBatchSliceFloats * 4;   // per-wavefront 16 x 16 product tile
    static constexpr size_t a_off = m_off + (size_t)16 * 256 * 4;           // G_n rows (FP16), pitch SP
    static constexpr size_t i_off = a_off + (size_t)kBatchMaxI * SP * 2;     // sample indices [CH][8]
    static constexpr size_t w_off = i_off + (size_t)CH * kMaxOrder * 4;      // weights [CH] float
    static constexpr size_t o_off = w_off + (size_t)CH * 4;                  // fiber offsets [CH] int64
    static constexpr size_t total = o_off + (size_t)CH * 8 + 64;
};

// SPLIT: one step of one sample range: workgroup b takes problem b / splits
// and the b % splits-th share of its chunks of samples, and writes its
// partial gradient (FP32, g[i * RR + c] at gpart + b * gstride) and its
// partial loss sum (lpart[b]) instead of updating the core; k_batch_apply
// then adds the shares and takes the step.  Otherwise workgroup b owns
// problem b for all ``steps`` steps.
template <int CH, int WAVES, bool SPLIT>
__global__ __launch_bounds__(64 * WAVES) void k_batch_steps(const tr_batch_item* __restrict__ items, int steps,
                                                            int splits, float* __restrict__ gpart,
                                                            double* __restrict__ lpart, int64_t gstride) {
    const int prob = SPLIT ? (int)blockIdx.x / splits : (int)blockIdx.x;
    const int share = SPLIT ? (int)blockIdx.x - prob * splits : 0;
    using Lz = BatchLds<CH>;
    constexpr int NT = 64 * WAVES;
    constexpr int RTW = 8 / WAVES;                           // row tiles of E per wavefront
    constexpr int GSL = (8 * 9 + WAVES - 1) / WAVES;       // g tiles per wavefront (MT <= 8, CT <= 9)
    constexpr int KS = kBatchMaxRR / 32;                     // K steps of the prediction GEMM
    // The problem's record in LDS: its sizes, ranks and core pointers are
    // indexed by mode at run time, which from global memory would cost a
    // dependent load per use.
    __shared__ __align__(16) tr_batch_item it;
    {
        const int* src = reinterpret_cast<const int*>(items + prob);
        int* dst = reinterpret_cast<int*>(&it);
        for (int i = threadIdx.x; i < (int)(sizeof(tr_batch_item) / 4); i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    const tr_desc& d = it.desc;
    const int N = d.N, tid = threadIdx.x, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int wv = tid >> 6;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    _Float16* sS = reinterpret_cast<_Float16*>(smem_raw + Lz::s_off);
    _Float16* sT = reinterpret_cast<_Float16*>(smem_raw + Lz::t_off);
    _Float16* sE = reinterpret_cast<_Float16*>(smem_raw + Lz::e_off);
    float* sC = reinterpret_cast<float*>(smem_raw + Lz::c_off);
    _Float16* sA = reinterpret_cast<_Float16*>(smem_raw + Lz::a_off);
    float* sM = reinterpret_cast<float*>(smem_raw + Lz::m_off);
    int* sidx = reinterpret_cast<int*>(smem_raw + Lz::i_off);
    float* sw = reinterpret_cast<float*>(smem_raw + Lz::w_off);
    int64_t* soff = reinterpret_cast<int64_t*>(smem_raw + Lz::o_off);
    __shared__ double red[WAVES];
    __shared__ int qoff[kMaxOrder + 1];   // slice offsets of the chain stages within a sample

    uint64_t t = *it.t_dev;
    const int m = it.m;
    for (int step = 0; step < steps; ++step) {
        const int n = pick_mode(it.seed, t, N);
        const int n1 = ring_next(n, N);
        const int In = d.I[n], Rn = d.R[n], Rn1 = d.R[n1], RR = Rn * Rn1;
        const int MT = (In + 15) >> 4, CT = (RR + 15) >> 4;
        const double J = (double)J_of(d, n);
        int64_t xs[kMaxOrder];                       // replica strides: fiber of mode n contiguous
        {
            int64_t s = In;
            xs[n] = 1;
            int k = n;
            for (int q = 1; q < N; ++q) {
                k = ring_next(k, N);
                xs[k] = s;
                s *= d.I[k];
            }
        }
        __syncthreads();   // the previous step is done with qoff
        if (tid == 0) {
            int o = 0;
            for (int q = 0; q < N - 1; ++q) {
                qoff[q] = o;
                const int k = (n + 1 + q) % N;
                o += d.R[k] * d.R[ring_next(k, N)];
            }
            qoff[N - 1] = o;
        }
        const float* Gn = static_cast<const float*>(it.cores[n]);
        const _Float16* X = static_cast<const _Float16*>(it.Xrep[n]);
        // G_n as FP16 A operands for the whole step (K padded with zeros);
        // loads at clamped indices, eight per thread in flight, masked after
        {
            constexpr int TOT = kBatchMaxI * kBatchMaxRR, UB = 8;
            for (int e0 = 0; e0 < TOT; e0 += NT * UB) {
                float gv[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = e0 + u * NT + tid;
                    const int row = e / kBatchMaxRR, k = e - row * kBatchMaxRR;
                    gv[u] = Gn[(int64_t)(row < In ? row : In - 1) * RR + (k < RR ? k : RR - 1)];
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = e0 + u * NT + tid;
                    const int row = e / kBatchMaxRR, k = e - row * kBatchMaxRR;
                    if (e < TOT) sA[row * Lz::SP + k] = (_Float16)((row < In && k < RR) ? gv[u] : 0.f);
                }
            }
        }
        f32x4b gacc[GSL];
#pragma unroll
        for (int q = 0; q < GSL; ++q) gacc[q] = f32x4b{0.f, 0.f, 0.f, 0.f};
        double lsum = 0.0;
        int fbeg = 0, fend = m;
        if (SPLIT) {   // this workgroup's share of the chunks
            const int nch = (m + CH - 1) / CH, cps = (nch + splits - 1) / splits;
            fbeg = min(m, share * cps * CH);
            fend = min(m, (share + 1) * cps * CH);
        }
        for (int f0 = fbeg; f0 < fend; f0 += CH) {
            const int nb = min(CH, m - f0);
            __syncthreads();   // previous chunk done with S, E, indices; qoff written
            for (int w = tid; w < nb * (N - 1); w += NT) {
                const int fl = w / (N - 1), q = w - fl * (N - 1);
                const int k = (n + 1 + q) % N;
                const uint64_t r = draw_word(it.seed, t, (uint64_t)(f0 + fl), (uint64_t)k, TR_STREAM_IDX);
                sidx[fl * kMaxOrder + k] = (int)mulhi64(r, (uint64_t)d.I[k]);
            }
            __syncthreads();
            for (int fl = tid; fl < CH; fl += NT) {
                float ws = 0.f;
                int64_t off = 0;
                if (fl < nb) {
                    double p = 1.0;   // uniform law, multiplied in the chain order
                    for (int q = 0; q < N - 1; ++q) {
                        const int k = (n + 1 + q) % N;
                        p = p * (1.0 / (double)d.I[k]);
                        off += (int64_t)sidx[fl * kMaxOrder + k] * xs[k];
                    }
                    ws = (float)(1.0 / (J * p));
                }
                sw[fl] = ws;
                soff[fl] = off;
            }
            // Rows of M_f = G_{n+1}(i) ... G_{n-1}(i), S(f, r + R_n s) = M_f(s, r),
            // kBatchGroup samples at a time: each slice is staged in LDS
            // zero-padded to 12 x 12 (element (r, c) at r + 12 c), every load
            // of the group in flight together; then one thread per (sample,
            // row s) carries row s of M_f through the chain in registers with
            // unrolled 12 x 12 products (the padding multiplies zeros).  FP32
            // throughout, rounded to FP16 once.
            constexpr int PS = kBatchRank * kBatchRank;                 // padded slice
            constexpr int PW = (kBatchGroup * (kBatchMaxN - 1) + WAVES - 1) / WAVES;   // slices per wave
            for (int g0 = 0; g0 < CH; g0 += kBatchGroup) {
                const int gn = min(kBatchGroup, CH - g0);
                float v[PW][3];
#pragma unroll
                for (int j = 0; j < PW; ++j) {
                    const int pr = wv + WAVES * j;                       // (sample, stage) pair
                    const int fl = pr / (N - 1), q = pr - fl * (N - 1);
                    int k = n + 1 + q;
                    k = k >= N ? k - N : k;
                    k = k >= N ? k - N : k;
                    const bool ok = pr < gn * (N - 1) && g0 + fl < nb;
                    const int Rk = d.R[k], Rk1 = d.R[k + 1 == N ? 0 : k + 1];
                    const float* src = static_cast<const float*>(it.cores[k]) +
                                       (int64_t)(ok ? sidx[(g0 + fl) * kMaxOrder + k] : 0) * Rk * Rk1;
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int pidx = l + 64 * u, r = pidx % kBatchRank, c = pidx / kBatchRank;
                        v[j][u] = src[(r < Rk ? r : Rk - 1) + Rk * (c < Rk1 ? c : Rk1 - 1)];
                    }
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int pidx = l + 64 * u, r = pidx % kBatchRank, c = pidx / kBatchRank;
                        if (!(ok && pidx < PS && r < Rk && c < Rk1)) v[j][u] = 0.f;
                    }
                }
#pragma unroll
                for (int j = 0; j < PW; ++j) {
                    const int pr = wv + WAVES * j;
                    if (pr < gn * (N - 1)) {
#pragma unroll
                        for (int u = 0; u < 3; ++u)
                            if (l + 64 * u < PS) sC[(size_t)pr * PS + l + 64 * u] = v[j][u];
                    }
                }
                __syncthreads();
                // chain products on FP32 matrix cores, one wavefront per
                // sample: M_q = M_{q-1} A_q as a 16 x 16 (zero-padded) tile,
                // K = 12 in three steps of 4; M_q goes back through this
                // wavefront's LDS tile to become the next A operand.
                float* Mw = sM + wv * 256;   // 16 x 16, row-major
                for (int fl = wv; fl < gn; fl += WAVES) {
                    const float* base = sC + (size_t)fl * (N - 1) * PS;
                    f32x4b m = {0.f, 0.f, 0.f, 0.f};
                    for (int q = 1; q < N - 1; ++q) {
                        const float* Aq = base + q * PS;
                        f32x4b acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int ks = 0; ks < 3; ++ks) {
                            const int kk = 4 * ks + lk;   // K index of this lane
                            // operands read at clamped indices and masked by a factor
                            // (a select would put each LDS read behind a branch)
                            const int lrc = lr < kBatchRank ? lr : kBatchRank - 1;
                            const float msk = lr < kBatchRank ? 1.f : 0.f;
                            float a;
                            if (q == 1) a = base[lrc + kBatchRank * kk] * msk;   // slice 0 (row lr)
                            else a = Mw[lr * 16 + kk];
                            const float b = Aq[kk + kBatchRank * lrc] * msk;
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
                        }
                        m = acc;
                        if (q + 1 < N - 1) {   // D rows 4 lk + j, column lr
                            __builtin_amdgcn_wave_barrier();
#pragma unroll
                            for (int j = 0; j < 4; ++j) Mw[(4 * lk + j) * 16 + lr] = m[j];
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                            __builtin_amdgcn_s_waitcnt(0xc07f);
                            __builtin_amdgcn_wave_barrier();
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        }
                    }
                    const int f = g0 + fl;
                    if (N == 2) {   // M_f is slice 0
#pragma unroll
                        for (int j = 0; j < 4; ++j) m[j] = (4 * lk + j < kBatchRank && lr < kBatchRank)
                                                               ? base[(4 * lk + j) + kBatchRank * lr] : 0.f;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int srow = 4 * lk + j, r = lr;   // M_f(srow, r) -> S(f, r + R_n srow)
                        if (srow < Rn1 && r < Rn) {
                            const _Float16 h = (_Float16)(f < nb ? m[j] : 0.f);
                            sS[f * Lz::SP + r + Rn * srow] = h;
                            sT[(r + Rn * srow) * Lz::TP + f] = h;
                        }
                    }
                }
                __syncthreads();   // slices consumed before the next group overwrites them
            }
            for (int w = tid; w < CH * (kBatchMaxRR - RR); w += NT) {   // K padding of S rows
                const int fl = w / (kBatchMaxRR - RR), c = RR + w % (kBatchMaxRR - RR);
                sS[fl * Lz::SP + c] = (_Float16)0.f;
            }
            for (int w = tid; w < (16 * CT - RR) * CH; w += NT) {        // column padding of S^T
                const int c = RR + w / CH, fl = w % CH;
                sT[c * Lz::TP + fl] = (_Float16)0.f;
            }
            __syncthreads();
            // E = X_F - G_n S^T: wavefront wv takes row tiles wv (+ WAVES),
            // all sample tiles; FP16 operands, FP32 accumulation.  The fiber
            // entries of the wavefront's outputs are loaded first (clamped
            // rows, all in flight) so no load waits inside the products.
            float xe[RTW][CH / 16][4];
#pragma unroll
            for (int u = 0; u < RTW; ++u)
#pragma unroll
                for (int st = 0; st < CH / 16; ++st) {
                    const int64_t off = soff[16 * st + lr];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int i = 16 * (wv + WAVES * u) + 4 * lk + j;
                        xe[u][st][j] = (float)X[off + (i < In ? i : In - 1)];
                    }
                }
#pragma unroll
            for (int u = 0; u < RTW; ++u) {
                const int rt = wv + WAVES * u;
#pragma unroll
                for (int st = 0; st < CH / 16; ++st) {
                    f32x4b acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        const h8 a = *reinterpret_cast<const h8*>(sA + (16 * rt + lr) * Lz::SP + 32 * ks + 8 * lk);
                        const h8 b = *reinterpret_cast<const h8*>(sS + (16 * st + lr) * Lz::SP + 32 * ks + 8 * lk);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
                    }
                    if (rt < MT) {
                        const int fl = 16 * st + lr;
                        const float ws = sw[fl];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int i = 16 * rt + 4 * lk + j;
                            float e = 0.f;
                            if (i < In && fl < nb) {
                                e = xe[u][st][j] - acc[j];
                                lsum += (double)ws * (double)e * (double)e;
                            }
                            sE[i * Lz::TP + fl] = (_Float16)(e * ws);
                        }
                    }
                }
            }
            __syncthreads();
            // g += (E D) S: tile T = wv + WAVES q of the MT x CT grid in slot q;
            // slots past the grid multiply zeros.
#pragma unroll
            for (int q = 0; q < GSL; ++q) {
                const int T = wv + WAVES * q;
                const bool ok = T < MT * CT;
                const int rt = ok ? T / CT : 0, ct = ok ? T - (T / CT) * CT : 0;
#pragma unroll
                for (int ks = 0; ks < CH / 32; ++ks) {
                    const int k0 = 32 * ks + 8 * lk;
                    const h8 a = ok ? *reinterpret_cast<const h8*>(sE + (16 * rt + lr) * Lz::TP + k0) : h8{};
                    const h8 b = ok ? *reinterpret_cast<const h8*>(sT + (16 * ct + lr) * Lz::TP + k0) : h8{};
                    gacc[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, gacc[q], 0, 0, 0);
                }
            }
        }
        if (SPLIT) {   // hand the partial sums to k_batch_apply
            float* gp = gpart + (int64_t)blockIdx.x * gstride;
#pragma unroll
            for (int q = 0; q < GSL; ++q) {
                const int T = wv + WAVES * q;
                if (T < MT * CT) {
                    const int rt = T / CT, ct = T - rt * CT;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int i = 16 * rt + 4 * lk + j, c = 16 * ct + lr;
                        if (i < In && c < RR) gp[(int64_t)i * RR + c] = gacc[q][j];
                    }
                }
            }
            const double ls = block_sum(lsum, red);
            if (tid == 0) lpart[blockIdx.x] = ls;
            return;
        }
        // p = g / m on this wavefront's tiles, then the rule
        float* G = static_cast<float*>(it.cores[n]);
        float* A = static_cast<float*>(it.accum[n]);
        const float invm = 1.f / (float)m;
        __syncthreads();   // every wavefront has read G_n for this step
#pragma unroll
        for (int q = 0; q < GSL; ++q) {
            const int T = wv + WAVES * q;
            if (T < MT * CT) {
                const int rt = T / CT, ct = T - rt * CT;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = 16 * rt + 4 * lk + j, c = 16 * ct + lr;
                    if (i < In && c < RR)
                        apply_rule<float>(G, A, (int64_t)i * RR + c, (double)(gacc[q][j] * invm), it.rule, t,
                                          it.dev_status);
                }
            }
        }
        // loss estimate sum_f ||e_f||^2 / (2 m p_f); lsum carries 1/(J p_f)
        const double ls = block_sum(lsum, red);
        if (tid == 0 && it.loss) *it.loss = ls * J / (2.0 * (double)m);
        t += 1;
        __syncthreads();   // the update is visible to the next step's reads (same workgroup)
    }
    if (tid == 0) *it.t_dev = t;
}

// The step of problem p after a split gradient: g = sum of the shares in
// share order, p = g / m (the sign of the direction folded in, as in the
// unsplit kernel), the rule on the core, the loss estimate, t + 1.
__global__ __launch_bounds__(1024) void k_batch_apply(const tr_batch_item* __restrict__ items, int splits,
                                                     const float* __restrict__ gpart,
                                                     const double* __restrict__ lpart, int64_t gstride) {
    const tr_batch_item& it = items[blockIdx.x];
    const tr_desc& d = it.desc;
    const uint64_t t = *it.t_dev;
    const int N = d.N;
    const int n = pick_mode(it.seed, t, N);
    const int In = d.I[n], RR = d.R[n] * d.R[ring_next(n, N)];
    const int m = it.m;
    const float invm = 1.f / (float)m;
    float* G = static_cast<float*>(it.cores[n]);
    float* A = static_cast<float*>(it.accum[n]);
    const float* gp = gpart + (int64_t)blockIdx.x * splits * gstride;
    // eight entries per thread per round, every load of the round in flight
    // (clamped indices), the shares added in order as before
    const int tot = In * RR;
    constexpr int U = 8;
    for (int e0 = 0; e0 < tot; e0 += (int)blockDim.x * U) {
        float g[U], gv[U], av[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x, ec = e < tot ? e : tot - 1;
            g[u] = 0.f;
            gv[u] = G[ec];
            av[u] = 0.f;
        }
        constexpr int QB = 4;   // shares fetched together
        for (int q0 = 0; q0 < splits; q0 += QB) {
            float pv[U][QB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x, ec = e < tot ? e : tot - 1;
#pragma unroll
                for (int qq = 0; qq < QB; ++qq) {
                    const int q = q0 + qq < splits ? q0 + qq : splits - 1;
                    pv[u][qq] = gp[(int64_t)q * gstride + ec];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int qq = 0; qq < QB; ++qq)
                    if (q0 + qq < splits) g[u] += pv[u][qq];
        }
        if (it.rule.kind == 1) {   // the accumulator exists only for AdaGrad
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x, ec = e < tot ? e : tot - 1;
                av[u] = A[ec];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x;
            if (e < tot) apply_rule_loaded<float>(G, A, e, gv[u], av[u], (double)(g[u] * invm), it.rule, t, it.dev_status);
        }
    }
    if (threadIdx.x == 0) {
        double ls = 0.0;
        for (int q = 0; q < splits; ++q) ls += lpart[(int64_t)blockIdx.x * splits + q];
        if (it.loss) *it.loss = ls * (double)J_of(d, n) / (2.0 * (double)m);
    }
    __syncthreads();   // every thread has read t
    if (threadIdx.x == 0) *it.t_dev = t + 1;
}

size_t batch_lds_bytes(int chunk) { return chunk == 32 ? BatchLds<32>::total : BatchLds<64>::total; }

size_t batch_split_ws_bytes(int count, int splits) {
    return align_up((size_t)count * splits * kBatchMaxI * kBatchMaxRR * 4) + align_up((size_t)count * splits * 8);
}

hipError_t launch_batch_split(const tr_batch_item* items, int count, int steps, int chunk, int waves, int splits,
                              void* ws, hipStream_t st) {
    const int64_t gstride = (int64_t)kBatchMaxI * kBatchMaxRR;
    float* gpart = static_cast<float*>(ws);
    double* lpart = reinterpret_cast<double*>(static_cast<char*>(ws) +
                                              align_up((size_t)count * splits * gstride * 4));
#define TRK_BSPLIT(CH, W)                                                                                   \
    do {                                                                                                    \
        const size_t shm = BatchLds<CH>::total;                                                            \
        if (!allow_lds(reinterpret_cast<const void*>(&k_batch_steps<CH, W, true>), shm))                  \
            return hipErrorInvalidValue;                                                                    \
        hipLaunchKernelGGL((k_batch_steps<CH, W, true>), dim3(count * splits), dim3(64 * W), shm, st, items, 1, \
                           splits, gpart, lpart, gstride);                                                  \
    } while (0)
    for (int s = 0; s < steps; ++s) {
        if (chunk == 32 && waves == 4) TRK_BSPLIT(32, 4);
        else if (chunk == 32 && waves == 8) TRK_BSPLIT(32, 8);
        else if (chunk == 64 && waves == 4) TRK_BSPLIT(64, 4);
        else if (chunk == 64 && waves == 8) TRK_BSPLIT(64, 8);
        else return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_batch_apply, dim3(count), dim3(1024), 0, st, items, splits, gpart, lpart, gstride);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
#undef TRK_BSPLIT
    return hipSuccess;
}

hipError_t launch_batch_steps(const tr_batch_item* items, int count, int steps, int chunk, int waves, hipStream_t st) {
#define TRK_BATCH(CH, W)                                                                                  \
    do {                                                                                                  \
        const size_t shm = BatchLds<CH>::total;                                                          \
        if (!allow_lds(reinterpret_cast<const void*>(&k_batch_steps<CH, W, false>), shm)) return hipErrorInvalidValue; \
        hipLaunchKernelGGL((k_batch_steps<CH, W, false>), dim3(count), dim3(64 * W), shm, st, items, steps, 1,   \
                           nullptr, nullptr, (int64_t)0);                                                 \
    } while (0)
    if (chunk == 32 && waves == 4) TRK_BATCH(32, 4);
    else if (chunk == 32 && waves == 8) TRK_BATCH(32, 8);
    else if (chunk == 64 && waves == 4) TRK_BATCH(64, 4);
    else if (chunk == 64 && waves == 8) TRK_BATCH(64, 8);
    else return hipErrorInvalidValue;
#undef TRK_BATCH
    return hipGetLastError();
}

}  // namespace trk
