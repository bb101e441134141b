// a7/a8: scaled direction p = -g (h + eta I)^{-1} by an FP64 Cholesky and
// two triangular solves (equation eq:scaledsg_direction and the amended
// preconditioner remark), then the step rule of eq:update_brsgd or the
// AdaGrad remark.
//
// The RR x RR factorisation is a serial chain of RR pivots: one block of
// 256 threads does it, in LDS when RR <= 128 (C3's 100 x 100 fits), else in
// the workspace.  If a pivot is not positive the factorisation restarts
// with eta + 10^(k-10) tr(h)/RR, k = 0..6.  The solves are independent per
// row of g: one wavefront per row, column-oriented substitution with the
// new unknown broadcast by a cross-lane shuffle.
#include "internal.hpp"

namespace trk {

// Right-looking lower Cholesky of the RR x RR matrix A (column-major, row
// pitch P, in LDS).  Pivot j: every thread reads the updated diagonal; the
// column below it is scaled by 1/L_jj (kept in dinv[j]; A's diagonal keeps
// L_jj^2) and copied to col[] (its own array, so the update's loads do not
// wait on its stores); then the trailing lower triangle takes the rank-1
// update, thread (r, ph) owning rows j+1+r (+64) and columns j+1+ph (+4),
// eight columns in flight at a time.  Two barriers per pivot; returns 1 (in
// every thread) at a pivot that is not positive.
__device__ inline int chol_lds(double* A, double* dinv, double* col, int RR, int P) {
    const int t = threadIdx.x, r = t & 63, ph = t >> 6;
    for (int j = 0; j < RR; ++j) {
        __syncthreads();
        const double djj = A[j + P * j];
        if (!(djj > 0.0) || !isfinite(djj)) return 1;
        const double inv = 1.0 / sqrt(djj);
        if (t == 0) dinv[j] = inv;
        for (int i = j + 1 + t; i < RR; i += 256) {
            const double v = A[i + P * j] * inv;
            A[i + P * j] = v;
            col[i] = v;
        }
        __syncthreads();
        for (int i = j + 1 + r; i < RR; i += 64) {
            const double lij = col[i];
            int k = j + 1 + ph;
            for (; k + 28 <= i; k += 32) {
                double a[8], c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    a[u] = A[i + P * (k + 4 * u)];
                    c[u] = col[k + 4 * u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) A[i + P * (k + 4 * u)] = a[u] - lij * c[u];
            }
            for (; k <= i; k += 4) A[i + P * k] -= lij * col[k];
        }
    }
    __syncthreads();
    return 0;
}

// Blocked right-looking Cholesky (16-column panels) of the RR x RR matrix A
// (column-major, pitch P, in LDS, RR <= 128), 256 threads.  Per panel:
//   1. wavefront 0 factors the 16 x 16 diagonal block in registers, lane i
//      holding row i; pivots and column entries are broadcast through the
//      scalar unit (no barrier inside the panel);
//   2. the rows below solve against it (one row per thread, 16 unknowns);
//   3. the trailing lower triangle takes the rank-16 update, thread (r, ph)
//      owning rows c0+16+r (+64) and columns c0+16+ph (+4).
// Three barriers per panel instead of two per column.  The diagonal of A keeps
// L_jj^2; dinv[j] = 1/L_jj.  Returns 1 in every thread on a pivot that is
// not positive.
__device__ inline int chol_blocked(double* A, double* dinv, int RR, int P) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    __shared__ int bad;
    for (int c0 = 0; c0 < RR; c0 += 16) {
        const int nb = min(16, RR - c0);
        if (wv == 0) {
            double dr[16];
#pragma unroll
            for (int k = 0; k < 16; ++k)
                dr[k] = (lane < nb && k <= lane) ? A[(c0 + lane) + P * (c0 + k)] : 0.0;
            int fail = 0;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                if (jj < nb) {
                    const double piv = readlane_f64(dr[jj], jj);
                    if (!(piv > 0.0) || !isfinite(piv)) fail = 1;
                    const double inv = 1.0 / sqrt(piv);
                    if (lane > jj) dr[jj] *= inv;
                    if (lane == jj) dinv[c0 + jj] = inv;
#pragma unroll
                    for (int kk = jj + 1; kk < 16; ++kk) {
                        if (kk < nb) {
                            const double lkj = readlane_f64(dr[jj], kk);
                            if (lane >= kk) dr[kk] -= dr[jj] * lkj;
                        }
                    }
                }
            }
            if (lane < nb) {
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    if (k <= lane) A[(c0 + lane) + P * (c0 + k)] = dr[k];
            }
            if (lane == 0) bad = fail;
        }
        __syncthreads();
        if (bad) return 1;
        for (int i = c0 + nb + t; i < RR; i += 256) {     // rows below: x L_D^T = a
            double x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) x[u] = u < nb ? A[i + P * (c0 + u)] : 0.0;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                if (jj < nb) {
                    double v = x[jj];
#pragma unroll
                    for (int kk = 0; kk < jj; ++kk) v -= x[kk] * A[(c0 + jj) + P * (c0 + kk)];
                    x[jj] = v * dinv[c0 + jj];
                }
            }
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (u < nb) A[i + P * (c0 + u)] = x[u];
        }
        __syncthreads();
        for (int i = c0 + nb + lane; i < RR; i += 64) {   // trailing rank-16 update
            double li[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) li[u] = u < nb ? A[i + P * (c0 + u)] : 0.0;
            for (int k = c0 + nb + wv; k <= i; k += 4) {
                double acc = A[i + P * k];
#pragma unroll
                for (int u = 0; u < 16; ++u) acc -= li[u] * (u < nb ? A[k + P * (c0 + u)] : 0.0);
                A[i + P * k] = acc;
            }
        }
        __syncthreads();
    }
    return 0;
}

// Factorise gram + eta I with the fallback ladder.  Lout: L below the
// diagonal (column-major, pitch RR), dinv_out: 1/L_jj; flag: 0 ok,
// 1 damped, 2 failed.
// USE_LDS is a template parameter: a pointer that may point to either LDS or
// global memory at run time compiles to flat (generic) accesses, which are
// far slower than LDS instructions.
template <bool USE_LDS>
__global__ __launch_bounds__(256) void k_chol(tr_desc d, ModeSrc ms, const double* __restrict__ gram,
                                              Damp dmp, double* __restrict__ Lout,
                                              double* __restrict__ dinv_out, int* __restrict__ flag,
                                              int32_t* status) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const double damping = dmp.at(t);
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = USE_LDS ? RR + 1 : RR;
    double* A = USE_LDS ? reinterpret_cast<double*>(smem_raw) : Lout;
    double* dinv = USE_LDS ? A + (size_t)P * RR : dinv_out;
    double* col = USE_LDS ? dinv + RR : dinv_out + RR;
    const int tid = threadIdx.x, r = tid & 63, ph = tid >> 6;
    __shared__ double red[4];
    double tr = 0.0;
    for (int c = tid; c < RR; c += 256) tr += gram[(int64_t)c * RR + c];
    const double base = (block_sum(tr, red) + damping * RR) / RR;   // tr(h + damping I) / RR
    int ok_at = -1;
    for (int attempt = 0; attempt < 8; ++attempt) {
        const double eta = attempt == 0 ? damping : damping + pow(10.0, (double)(attempt - 1 - 10)) * base;
        __syncthreads();
        if (USE_LDS) {   // RR <= 128: every load of the fill issued before any store
            double v[32][2];
#pragma unroll
            for (int a = 0; a < 32; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int k = ph + 4 * a, c = r + 64 * b;
                    v[a][b] = (k < RR && c < RR) ? gram[(int64_t)k * RR + c] : 0.0;
                }
#pragma unroll
            for (int a = 0; a < 32; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int k = ph + 4 * a, c = r + 64 * b;
                    if (k < RR && c < RR) A[c + P * k] = v[a][b] + (c == k ? eta : 0.0);
                }
            __syncthreads();
            if (chol_blocked(A, dinv, RR, P) == 0) {
                ok_at = attempt;
                break;
            }
        } else {
            for (int k = ph; k < RR; k += 4)
                for (int c = r; c < RR; c += 64)
                    A[c + (int64_t)P * k] = gram[(int64_t)k * RR + c] + (c == k ? eta : 0.0);
            if (chol_lds(A, dinv, col, RR, P) == 0) {
                ok_at = attempt;
                break;
            }
        }
    }
    __syncthreads();
    if (USE_LDS) {
        for (int k = ph; k < RR; k += 4)
            for (int c = r; c < RR; c += 64) Lout[c + (int64_t)RR * k] = A[c + (int64_t)P * k];
        for (int j = tid; j < RR; j += 256) dinv_out[j] = dinv[j];
    }
    if (tid == 0) {
        const int fl = ok_at < 0 ? 2 : (ok_at > 0 ? 1 : 0);
        *flag = fl;
        if (fl == 1) set_status(status, TR_DEV_DAMPED);
        if (fl == 2) set_status(status, TR_DEV_NOT_SPD);
    }
}

constexpr int kSolveWaves = 16;

// p_i = -(L L^T)^{-1} g_i^T for every row i of g, then the rule.  L is staged
// in LDS once per block (odd pitch: both the column reads of the forward
// solve and the row reads of the backward solve avoid bank conflicts).  Each
// wavefront solves one row: column-oriented substitution; the new unknown is
// scaled by its reciprocal pivot on the lane that owns it and broadcast
// through the scalar unit; the L entries a step needs are loaded before the
// broadcast so the two latencies overlap.
template <typename TC, bool USE_LDS>
__global__ __launch_bounds__(1024) void k_solve_update(tr_desc d, ModeSrc ms, const TC* __restrict__ g,
                                                       const double* __restrict__ L,
                                                       const double* __restrict__ dinv,
                                                       const int* __restrict__ flag, MutPtrs cores,
                                                       MutPtrs accum, tr_step rule, int32_t* status) {
    constexpr bool use_lds = USE_LDS;
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    if (*flag == 2) return;            // not positive definite: core unchanged
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int P = use_lds ? RR + 1 : RR;
    double* lL = reinterpret_cast<double*>(smem_raw);
    if (use_lds) {   // RR <= 128: every load issued before any store
        double v[8][2];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int k = wv + kSolveWaves * a, c = lane + 64 * b;
                v[a][b] = (k < RR && c < RR) ? L[c + (int64_t)RR * k] : 0.0;
            }
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int k = wv + kSolveWaves * a, c = lane + 64 * b;
                if (k < RR && c < RR) lL[c + P * k] = v[a][b];
            }
        __syncthreads();
    }
    const double* sL = use_lds ? lL : L;   // too large for LDS: read through the caches
    constexpr int Q = kMaxRR / 64;     // entries per lane
    double dv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int c = lane + 64 * q;
        dv[q] = c < RR ? dinv[c] : 0.0;
    }
    TC* G = static_cast<TC*>(cores.p[n]);
    TC* A = static_cast<TC*>(accum.p[n]);
    for (int row = blockIdx.x * kSolveWaves + wv; row < In; row += gridDim.x * kSolveWaves) {
        double y[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = lane + 64 * q;
            y[q] = c < RR ? (double)g[(int64_t)row * RR + c] : 0.0;
        }
        for (int j = 0; j < RR; ++j) {          // L z = g
            const int qj = j >> 6, lj = j & 63;
            double lc[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int c = lane + 64 * q;
                lc[q] = (c > j && c < RR) ? sL[c + P * j] : 0.0;
            }
            double own = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (q == qj) own = y[q] * dv[q];
            const double zj = readlane_f64(own, lj);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int c = lane + 64 * q;
                y[q] = c == j ? zj : y[q] - lc[q] * zj;
            }
        }
        for (int j = RR - 1; j >= 0; --j) {     // L^T x = z
            const int qj = j >> 6, lj = j & 63;
            double lc[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int c = lane + 64 * q;
                lc[q] = c < j ? sL[j + P * c] : 0.0;
            }
            double own = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (q == qj) own = y[q] * dv[q];
            const double xj = readlane_f64(own, lj);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int c = lane + 64 * q;
                y[q] = c == j ? xj : y[q] - lc[q] * xj;
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = lane + 64 * q;
            if (c < RR) apply_rule<TC>(G, A, (int64_t)row * RR + c, -y[q], rule, t, status);
        }
    }
}

template <typename TC>
__global__ __launch_bounds__(256) void k_plain_update(tr_desc d, ModeSrc ms, const TC* __restrict__ g,
                                                      MutPtrs cores, MutPtrs accum, tr_step rule,
                                                      int32_t* status) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int64_t total = (int64_t)d.I[n] * d.R[n] * d.R[ring_next(n, d.N)];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    TC* G = static_cast<TC*>(cores.p[n]);
    TC* A = static_cast<TC*>(accum.p[n]);
    apply_rule<TC>(G, A, e, -(double)g[e], rule, t, status);
}

UpdWs upd_ws_layout(const tr_desc& d) {
    UpdWs L{};
    const Shape sh = shape_of(d);
    L.L_off = 0;
    L.dinv_off = align_up((size_t)sh.maxRR * sh.maxRR * 8);
    L.flag_off = L.dinv_off + align_up((size_t)sh.maxRR * 16);   // dinv + column buffer
    L.total = L.flag_off + 256;
    return L;
}

hipError_t launch_scaled_update(const tr_desc& d, ModeSrc ms, const double* gram, Damp damping, const void* g,
                                MutPtrs cores, MutPtrs accum, tr_step rule, int32_t* status, void* ws,
                                const UpdWs& L, hipStream_t st) {
    if (sweep_supported(d))
        return launch_sweep_update(d, ms, gram, damping, g, nullptr, cores, accum, rule, status, ws, L, StepBump{},
                                   st);
    const Shape sh = shape_of(d);
    char* w = static_cast<char*>(ws);
    double* Lm = reinterpret_cast<double*>(w + L.L_off);
    double* dinv = reinterpret_cast<double*>(w + L.dinv_off);
    int* flag = reinterpret_cast<int*>(w + L.flag_off);
    const size_t want = ((size_t)(sh.maxRR + 1) * sh.maxRR + 2 * sh.maxRR) * 8;
    if (sh.maxRR <= 128 && allow_lds(reinterpret_cast<const void*>(&k_chol<true>), want))
        hipLaunchKernelGGL(k_chol<true>, dim3(1), dim3(256), want, st, d, ms, gram, damping, Lm, dinv, flag, status);
    else
        hipLaunchKernelGGL(k_chol<false>, dim3(1), dim3(256), 0, st, d, ms, gram, damping, Lm, dinv, flag, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((sh.maxI + kSolveWaves - 1) / kSolveWaves);
    const size_t want_s = (size_t)(sh.maxRR + 1) * sh.maxRR * 8;
#define TRK_SOLVE(TC)                                                                                       \
    if (sh.maxRR <= 128 && allow_lds(reinterpret_cast<const void*>(&k_solve_update<TC, true>), want_s))                          \
        hipLaunchKernelGGL((k_solve_update<TC, true>), grid, dim3(64 * kSolveWaves), want_s, st, d, ms,       \
                           static_cast<const TC*>(g), Lm, dinv, flag, cores, accum, rule, status);           \
    else                                                                                                     \
        hipLaunchKernelGGL((k_solve_update<TC, false>), grid, dim3(64 * kSolveWaves), 0, st, d, ms,           \
                           static_cast<const TC*>(g), Lm, dinv, flag, cores, accum, rule, status)
    if (d.core_dtype == TR_F64) {
        TRK_SOLVE(double);
    } else {
        TRK_SOLVE(float);
    }
#undef TRK_SOLVE
    return hipGetLastError();
}

hipError_t launch_plain_update(const tr_desc& d, ModeSrc ms, const void* g, MutPtrs cores, MutPtrs accum,
                               tr_step rule, int32_t* status, hipStream_t st) {
    const Shape sh = shape_of(d);
    const dim3 grid((unsigned)(((int64_t)sh.maxI * sh.maxRR + 255) / 256));
    if (d.core_dtype == TR_F64)
        hipLaunchKernelGGL(k_plain_update<double>, grid, dim3(256), 0, st, d, ms, static_cast<const double*>(g),
                           cores, accum, rule, status);
    else
        hipLaunchKernelGGL(k_plain_update<float>, grid, dim3(256), 0, st, d, ms, static_cast<const float*>(g),
                           cores, accum, rule, status);
    return hipGetLastError();
}

}  // namespace trk
