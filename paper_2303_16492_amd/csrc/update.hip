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

__device__ inline int chol_inplace(double* A, int RR) {
    // Right-looking lower Cholesky on column-major A; returns 0 on success.
    __shared__ int fail;
    for (int j = 0; j < RR; ++j) {
        __syncthreads();
        const double djj = A[j + (int64_t)RR * j];
        if (!(djj > 0.0) || !isfinite(djj)) return 1;   // same value in every thread
        const double ljj = sqrt(djj);
        __syncthreads();
        for (int i = j + threadIdx.x; i < RR; i += blockDim.x)
            A[i + (int64_t)RR * j] = i == j ? ljj : A[i + (int64_t)RR * j] / ljj;
        __syncthreads();
        const int w = RR - j - 1;
        for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
            const int i = j + 1 + e % w, k = j + 1 + e / w;
            if (k <= i) A[i + (int64_t)RR * k] -= A[i + (int64_t)RR * j] * A[k + (int64_t)RR * j];
        }
    }
    (void)fail;
    __syncthreads();
    return 0;
}

// Factorise gram + eta I with the fallback ladder; L (lower, column-major)
// goes to Lout, flag: 0 ok, 1 damped, 2 failed.
__global__ __launch_bounds__(256) void k_chol(tr_desc d, ModeSrc ms, const double* __restrict__ gram,
                                              double damping, double* __restrict__ Lout,
                                              int* __restrict__ flag, int32_t* status, int use_lds) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* A = use_lds ? reinterpret_cast<double*>(smem_raw) : Lout;
    __shared__ double trace_s;
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int c = 0; c < RR; ++c) tr += gram[(int64_t)c * RR + c];
        trace_s = tr + damping * RR;   // trace of the damped h
    }
    __syncthreads();
    const double base = trace_s / RR;
    int ok_at = -1;
    for (int attempt = 0; attempt < 8; ++attempt) {
        const double eta = attempt == 0 ? damping : damping + pow(10.0, (double)(attempt - 1 - 10)) * base;
        __syncthreads();
        for (int e = threadIdx.x; e < RR * RR; e += blockDim.x) {
            const int c = e % RR, k = e / RR;   // column-major (c row, k col); gram is symmetric
            A[e] = gram[(int64_t)k * RR + c] + (c == k ? eta : 0.0);
        }
        if (chol_inplace(A, RR) == 0) {
            ok_at = attempt;
            break;
        }
    }
    __syncthreads();
    if (use_lds)
        for (int e = threadIdx.x; e < RR * RR; e += blockDim.x) Lout[e] = A[e];
    if (threadIdx.x == 0) {
        const int fl = ok_at < 0 ? 2 : (ok_at > 0 ? 1 : 0);
        *flag = fl;
        if (fl == 1) set_status(status, TR_DEV_DAMPED);
        if (fl == 2) set_status(status, TR_DEV_NOT_SPD);
    }
}

// One wavefront per row i of g: p_i = -(L L^T)^{-1} g_i^T, then the rule.
template <typename TC>
__global__ __launch_bounds__(256) void k_solve_update(tr_desc d, ModeSrc ms, const TC* __restrict__ g,
                                                      const double* __restrict__ L,
                                                      const int* __restrict__ flag, MutPtrs cores,
                                                      MutPtrs accum, tr_step rule, int32_t* status) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const int In = d.I[n];
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= In) return;
    if (*flag == 2) return;            // not positive definite: core unchanged
    constexpr int Q = kMaxRR / 64;     // entries per lane
    double y[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int c = lane + 64 * q;
        y[q] = c < RR ? (double)g[(int64_t)row * RR + c] : 0.0;
    }
    // forward: L z = g
    for (int j = 0; j < RR; ++j) {
        const int qj = j >> 6, lj = j & 63;
        double yj = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (q == qj) yj = y[q];
        yj = __shfl(yj, lj, 64) / L[j + (int64_t)RR * j];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = lane + 64 * q;
            if (c == j) y[q] = yj;
            else if (c > j && c < RR) y[q] -= L[c + (int64_t)RR * j] * yj;
        }
    }
    // backward: L^T x = z
    for (int j = RR - 1; j >= 0; --j) {
        const int qj = j >> 6, lj = j & 63;
        double xj = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (q == qj) xj = y[q];
        xj = __shfl(xj, lj, 64) / L[j + (int64_t)RR * j];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = lane + 64 * q;
            if (c == j) y[q] = xj;
            else if (c < j) y[q] -= L[j + (int64_t)RR * c] * xj;
        }
    }
    TC* G = static_cast<TC*>(cores.p[n]);
    TC* A = static_cast<TC*>(accum.p[n]);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int c = lane + 64 * q;
        if (c < RR) {
            const int64_t e = (int64_t)row * RR + c;
            apply_rule<TC>(G, A, e, -y[q], rule, t, status);
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
    L.flag_off = align_up((size_t)sh.maxRR * sh.maxRR * 8);
    L.total = L.flag_off + 256;
    return L;
}

hipError_t launch_scaled_update(const tr_desc& d, ModeSrc ms, const double* gram, double damping, const void* g,
                                MutPtrs cores, MutPtrs accum, tr_step rule, int32_t* status, void* ws,
                                const UpdWs& L, hipStream_t st) {
    const Shape sh = shape_of(d);
    char* w = static_cast<char*>(ws);
    double* Lm = reinterpret_cast<double*>(w + L.L_off);
    int* flag = reinterpret_cast<int*>(w + L.flag_off);
    const size_t want = (size_t)sh.maxRR * sh.maxRR * 8;
    const int use_lds = (sh.maxRR <= 128 && allow_lds(reinterpret_cast<const void*>(&k_chol), want)) ? 1 : 0;
    const size_t shm = use_lds ? want : 0;
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), shm, st, d, ms, gram, damping, Lm, flag, status, use_lds);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((sh.maxI + 3) / 4);
    if (d.core_dtype == TR_F64)
        hipLaunchKernelGGL(k_solve_update<double>, grid, dim3(256), 0, st, d, ms, static_cast<const double*>(g),
                           Lm, flag, cores, accum, rule, status);
    else
        hipLaunchKernelGGL(k_solve_update<float>, grid, dim3(256), 0, st, d, ms, static_cast<const float*>(g), Lm,
                           flag, cores, accum, rule, status);
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
