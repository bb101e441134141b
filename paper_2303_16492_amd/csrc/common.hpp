// Shared device/host helpers of the gfx950 tensor-ring library.
//
// Random draws: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and
// Lemire's bounded integers floor(r * n / 2^64) (ACM TOMACS 2019).
// Layouts and index conventions are those of include/tr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "tr.h"

namespace trk {

constexpr int kMaxOrder = TR_MAX_ORDER;
constexpr int kMaxRank = TR_MAX_RANK;
constexpr int kMaxRR = kMaxRank * kMaxRank;

// ------------------------------------------------------------------ RNG --

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

// First output word of one Philox4x64-10 block, key (seed, 0).
__host__ __device__ inline uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t c3, uint64_t seed) {
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t lo0 = kPhiloxM0 * c0, hi0 = mulhi64(kPhiloxM0, c0);
        const uint64_t lo1 = kPhiloxM1 * c2, hi1 = mulhi64(kPhiloxM1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return c0;
}

__host__ __device__ inline uint64_t draw_word(uint64_t seed, uint64_t t, uint64_t f, uint64_t k,
                                              uint64_t stream) {
    return philox_word0(t, f, k, stream, seed);
}

__host__ __device__ inline int pick_mode(uint64_t seed, uint64_t t, int N) {
    return (int)mulhi64(draw_word(seed, t, 0, 0, TR_STREAM_MODE), (uint64_t)N);
}

// Integer-CDF pick: first i with cdf[i] > u, u = floor(r * W / 2^64).
template <typename P>
__device__ inline int cdf_pick(P cdf, int len, uint64_t r, double* p) {
    const uint64_t W = cdf[len - 1];
    const uint64_t u = mulhi64(r, W);
    int lo = 0, hi = len - 1;           // answer in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    const uint64_t prev = lo > 0 ? cdf[lo - 1] : 0ull;
    *p = (double)(cdf[lo] - prev) / (double)W;
    return lo;
}

// ---------------------------------------------------------------- modes --

// Where a kernel takes its step index and mode from: a device counter
// (graph-replayable runs) or host values.
struct ModeSrc {
    const uint64_t* t_dev;   // if non-null, t = *t_dev
    uint64_t t;
    int32_t n;               // >= 0: this mode; -1: pick_mode(seed, t, N); -2: *n_dev
    uint64_t seed;
    const int32_t* n_dev;    // the mode of the step, published by its first kernel (n == -2)
    int32_t* n_pub;          // n == -1: where the step's first kernel publishes the mode it drew
};

// Damping eta^t of the amended preconditioner h + eta^t I (the remark after
// eq:scaledsg_direction): kind 0 constant eta0, 1 harmonic eta0 / (1 + t/tau),
// 2 geometric eta0 tau^t.  A plain double converts to the constant kind.
struct Damp {
    double eta0 = 0.0, tau = 1.0;
    int32_t kind = 0;
    Damp() = default;
    __host__ __device__ Damp(double e) : eta0(e) {}
    __host__ __device__ Damp(double e, double ta, int32_t k) : eta0(e), tau(ta), kind(k) {}
    __host__ __device__ double at(uint64_t t) const {
        if (kind == 1) return eta0 / (1.0 + (double)t / tau);
        if (kind == 2) return eta0 * pow(tau, (double)t);
        return eta0;
    }
};

// The two loads (step counter, published mode) are independent, so a
// kernel that needs both waits for one memory round trip.
__device__ inline void resolve_mode(const ModeSrc& ms, int N, uint64_t* t, int* n) {
    const uint64_t tt = ms.t_dev ? *ms.t_dev : ms.t;
    *t = tt;
    *n = ms.n >= 0 ? ms.n : (ms.n == -2 ? *ms.n_dev : pick_mode(ms.seed, tt, N));
}

struct Ptrs {
    const void* p[kMaxOrder];
};
struct MutPtrs {
    void* p[kMaxOrder];
};
struct CdfPtrs {
    const uint64_t* p[kMaxOrder];
};

__host__ __device__ inline int ring_next(int k, int N) { return k + 1 == N ? 0 : k + 1; }

// Entry k of a per-mode kernel-argument table where k differs between the
// lanes of a wavefront.  Indexing the table directly would be a per-lane
// vector load from the argument segment (a memory round trip, and its wait
// also drains every store issued before it); the unrolled selects take all
// entries from scalar registers.
// (The empty asm makes each entry an opaque scalar value; without it the
// compiler folds the selects back into one indexed load.)
template <typename T>
__device__ inline T lane_pick(const T (&tab)[kMaxOrder], int k) {
    T r = tab[0];
    asm("" : "+s"(r));
#pragma unroll
    for (int j = 1; j < kMaxOrder; ++j) {
        T e = tab[j];
        asm("" : "+s"(e));
        r = k == j ? e : r;
    }
    return r;
}

// Pointer in global memory (an opaque pointer has lost the address space the
// compiler infers for kernel arguments; a generic one would make every load
// through it a flat load).
template <typename T>
using gptr = const T __attribute__((address_space(1)))*;

template <typename T, typename P>
__device__ inline gptr<T> lane_pick_global(const P (&tab)[kMaxOrder], int k) {
    return (gptr<T>)(const T*)lane_pick(tab, k);
}

__host__ __device__ inline int64_t J_of(const tr_desc& d, int n) {
    int64_t J = 1;
    for (int k = 0; k < d.N; ++k)
        if (k != n) J *= d.I[k];
    return J;
}

// Offset of the fiber of mode n through the sampled indices of row f.
__device__ inline int64_t fiber_base(const tr_desc& d, int n, const int32_t* __restrict__ idxrow) {
    int64_t off = 0;
    for (int k = 0; k < d.N; ++k)
        if (k != n) off += (int64_t)idxrow[k] * d.x_stride[k];
    return off;
}

// ---------------------------------------------------------------- types --

template <typename T> struct Cvt;
template <> struct Cvt<double> {
    __device__ static double to_f64(double v) { return v; }
    __device__ static float to_f32(double v) { return (float)v; }
};
template <> struct Cvt<float> {
    __device__ static double to_f64(float v) { return (double)v; }
    __device__ static float to_f32(float v) { return v; }
};
template <> struct Cvt<__half> {
    __device__ static double to_f64(__half v) { return (double)__half2float(v); }
    __device__ static float to_f32(__half v) { return __half2float(v); }
};
template <> struct Cvt<__hip_bfloat16> {
    __device__ static double to_f64(__hip_bfloat16 v) { return (double)__bfloat162float(v); }
    __device__ static float to_f32(__hip_bfloat16 v) { return __bfloat162float(v); }
};

template <typename T> __device__ inline T from_f64(double v);
template <> __device__ inline double from_f64<double>(double v) { return v; }
template <> __device__ inline float from_f64<float>(double v) { return (float)v; }
template <> __device__ inline __half from_f64<__half>(double v) { return __float2half((float)v); }
template <> __device__ inline __hip_bfloat16 from_f64<__hip_bfloat16>(double v) {
    return __float2bfloat16((float)v);
}

template <typename T> __device__ inline double to_f64(T v) { return Cvt<T>::to_f64(v); }

// ----------------------------------------------------------- reductions --

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum in a fixed order (waves then lanes); result valid in all
// threads.  ``scratch`` needs blockDim/64 entries.
template <typename T>
__device__ inline T block_sum(T v, T* scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < nw; ++w) s += scratch[w];
    __syncthreads();
    return s;
}

// Four consecutive tensor entries from a 4-element-aligned address.
__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
}
__device__ __forceinline__ void load4(const __half* p, float (&v)[4]) {
    const uint2 q = *reinterpret_cast<const uint2*>(p);
    const __half2 a = *reinterpret_cast<const __half2*>(&q.x), b = *reinterpret_cast<const __half2*>(&q.y);
    v[0] = __low2float(a);
    v[1] = __high2float(a);
    v[2] = __low2float(b);
    v[3] = __high2float(b);
}

__device__ inline void set_status(int32_t* st, int32_t bits) {
    if (st && bits) atomicOr(st, bits);
}

// Step rule for one core entry: eq:update_brsgd (fixed alpha), Robbins-Monro
// alpha_t = alpha/(1 + t/tau), or the AdaGrad remark (accumulator includes
// the current step; no change where b + A == 0).
// The same with the entry's current value ``old`` and AdaGrad accumulator
// ``acc_old`` already loaded (callers that fetch them early).
template <typename TC>
__device__ inline void apply_rule_loaded(TC* G, TC* A, int64_t e, double old, double acc_old, double p,
                                         const tr_step& rule, uint64_t t, int32_t* status) {
    double nv;
    if (rule.kind == 1) {
        const double a = acc_old + p * p;
        A[e] = (TC)a;
        const double base = rule.b + a;
        double stepm = 0.0;
        if (base > 0.0) stepm = rule.eta / (rule.eps == 0.0 ? sqrt(base) : pow(base, 0.5 + rule.eps));
        nv = old + stepm * p;
    } else if (rule.kind == 2) {
        nv = old + rule.alpha / (1.0 + (double)t / rule.tau) * p;
    } else {
        nv = old + rule.alpha * p;
    }
    if (!isfinite(nv)) set_status(status, TR_DEV_NONFINITE);
    G[e] = (TC)nv;
}

template <typename TC>
__device__ inline void apply_rule(TC* G, TC* A, int64_t e, double p, const tr_step& rule, uint64_t t,
                                  int32_t* status) {
    const double old = (double)G[e];
    double nv;
    if (rule.kind == 1) {
        const double a = (double)A[e] + p * p;
        A[e] = (TC)a;
        const double base = rule.b + a;
        double stepm = 0.0;
        if (base > 0.0) stepm = rule.eta / (rule.eps == 0.0 ? sqrt(base) : pow(base, 0.5 + rule.eps));
        nv = old + stepm * p;
    } else if (rule.kind == 2) {
        nv = old + rule.alpha / (1.0 + (double)t / rule.tau) * p;
    } else {
        nv = old + rule.alpha * p;
    }
    if (!isfinite(nv)) set_status(status, TR_DEV_NONFINITE);
    G[e] = (TC)nv;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Opt a kernel into more than 64 KiB of dynamic LDS (gfx950 has 160 KiB per
// CU).  Returns false if the runtime refuses; callers then take a path that
// needs less LDS or report the error.
inline bool allow_lds(const void* kernel, size_t bytes) {
    if (bytes <= 65536) return true;
    if (bytes > 160 * 1024) return false;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess) return true;
    (void)hipGetLastError();   // a refusal must not surface as a later launch error
    return false;
}

// Broadcast of a uniform lane's double through the scalar unit (no LDS
// round trip, unlike a shuffle).  ``lane`` must be the same in every lane.
__device__ inline double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace trk
