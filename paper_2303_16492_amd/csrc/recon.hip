// a9: full reconstruction X_hat_[1] = G_{1(2)} (G^{!=1}_[2])^T and the RSE of
// Section 4, ||X_hat - X_true||_F / ||X_true||_F, with FP64 sums.
//
// A block owns TJ columns j of X_[1] (paper order: column j is the
// multi-index of (i_2..i_N), first fastest).  It builds their subchain rows
// s_j in LDS (chain products, one thread per (column, row of M_j)), then
// every thread takes rows i_1 = tid, tid + 256, ... and forms the TJ dot
// products G_{1(2)}(i_1, :) . s_j with G streamed through registers and s_j
// broadcast from LDS.  X_true is read once, coalesced along i_1.  Per-block
// FP64 partial sums are added in a fixed order by a second kernel.
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

__global__ void k_recon_finish(const double* __restrict__ part, int64_t nblocks, double xnorm2, double* rse,
                               double* sums) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = 0.0, q = 0.0;
    for (int64_t b = 0; b < nblocks; ++b) {
        e += part[2 * b];
        q += part[2 * b + 1];
    }
    if (xnorm2 >= 0.0) q = xnorm2;
    sums[0] = e;
    sums[1] = q;
    *rse = sqrt(e) / sqrt(q);
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

size_t relerr_ws_bytes(const tr_desc& d) { return align_up(16) + align_up((size_t)recon_blocks(d) * 16); }

hipError_t launch_relerr(const tr_desc& d, Ptrs cores, const void* Xt, double xnorm2, double* rse, void* ws,
                         hipStream_t st) {
    const int64_t nb = recon_blocks(d);
    char* w = static_cast<char*>(ws);
    double* sums = reinterpret_cast<double*>(w);
    double* part = reinterpret_cast<double*>(w + align_up(16));
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
    hipLaunchKernelGGL(k_recon_finish, dim3(1), dim3(64), 0, st, part, nb, xnorm2, rse, sums);
    return hipGetLastError();
}

hipError_t launch_reconstruct(const tr_desc& d, Ptrs cores, void* Xo, hipStream_t st) {
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
