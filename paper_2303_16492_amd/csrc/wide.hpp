// Shared pieces of the 16-byte-operand gradient kernels (FP32 and 16-bit
// matrix cores): one chunk of 128 samples per sample group, the chunk's rows
// of S staged in LDS by direct memory-to-LDS loads, each sample's fiber
// offset and weights in lane order, and the per-mode constants computed on
// the host.
#pragma once
#include "internal.hpp"

namespace trk {

constexpr int kWideTF = 128;   // samples per chunk (one chunk per sample group)

// The 16-byte-operand kernels apply: one chunk of kWideTF samples per sample
// group, every R_n R_{n+1} a multiple of 4 with the largest in (32, 128], S,
// the cores and the partials 16-byte aligned.
inline bool wide_applies(const tr_desc& d, Ptrs cores, const float* S, const float* gp, int m, int groups,
                         int maxRR, int tf) {
    if (tf != kWideTF || (m + kWideTF - 1) / kWideTF > groups || maxRR <= 32 || maxRR > 128) return false;
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if (!al(S) || !al(gp)) return false;
    for (int k = 0; k < d.N; ++k) {
        if ((d.R[k] * d.R[(k + 1) % d.N]) % 4 != 0) return false;
        if (cores.p[k] && !al(cores.p[k])) return false;
    }
    return true;
}

// R_n R_{n+1} when every mode has the same (the chunk's loads then go out
// before the step's mode is known), else 0.
inline int wide_rr_fixed(const tr_desc& d) {
    int rr = d.R[0] * d.R[1 % d.N];
    for (int k = 1; k < d.N; ++k)
        if (d.R[k] * d.R[(k + 1) % d.N] != rr) rr = 0;
    return rr;
}

// What the kernels need of the step's mode, computed once on the host for
// every mode: the element stride of each index in the fiber source (zero
// for the mode itself, so an offset is the plain sum over all modes), the
// sample weight's factor 1/(m J_n), and whether fibers are contiguous whole
// 4-row groups at a 4-entry-aligned source.
struct WideMode {
    int64_t xs[kMaxOrder];
    double wbase;
    int32_t fast;
};
struct WideModes {
    WideMode md[kMaxOrder];
};

inline WideModes wide_modes(const tr_desc& d, XSrc xs, int m, size_t xelem) {
    WideModes tab{};
    for (int n = 0; n < d.N; ++n) {
        WideMode& md = tab.md[n];
        const void* src = xs.rep[n] ? xs.rep[n] : xs.X;
        int64_t xsn;
        if (xs.rep[n]) {   // mode-major replica: mode n fastest, then the ring order after n
            int64_t s = d.I[n];
            xsn = 1;
            for (int q = 1, k = n; q < d.N; ++q) {
                k = (k + 1) % d.N;
                md.xs[k] = s;
                s *= d.I[k];
            }
        } else {
            for (int k = 0; k < d.N; ++k) md.xs[k] = d.x_stride[k];
            xsn = d.x_stride[n];
        }
        md.xs[n] = 0;
        md.wbase = 1.0 / ((double)m * (double)J_of(d, n));
        md.fast = xsn == 1 && (d.I[n] & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & (4 * xelem - 1)) == 0;
    }
    return tab;
}

__device__ __forceinline__ float4 mask4(float4 v, bool ok) {
    const unsigned mk = ok ? 0xffffffffu : 0u;
    return make_float4(__uint_as_float(__float_as_uint(v.x) & mk), __uint_as_float(__float_as_uint(v.y) & mk),
                       __uint_as_float(__float_as_uint(v.z) & mk), __uint_as_float(__float_as_uint(v.w) & mk));
}

// Sum over a wavefront in a fixed order without LDS: pairs, quads, half
// rows and rows by DPP lane moves, then the four row sums read from lanes
// 0, 16, 32 and 48.  Valid in every lane.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_id) {
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    switch (ctrl_id) {
        case 0:   // quad_perm [1,0,3,2]
            lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
            break;
        case 1:   // quad_perm [2,3,0,1]
            lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
            break;
        case 2:   // row_half_mirror
            lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
            break;
        default:   // row_mirror
            lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false);
            break;
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_f64(v, 0);
    v += dpp_f64(v, 1);
    v += dpp_f64(v, 2);
    v += dpp_f64(v, 3);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Direct memory-to-LDS staging of the chunk's rows of S, 16 bytes a lane.
// LDS rows have Q pieces of 16 bytes; piece k of staged row f is piece
// f q0 + k of the chunk's rows in memory (q0 = R_n R_{n+1} / 4), so pieces
// past q0 continue into the next row and the staged area is a flat copy:
// piece e at byte 16 e.  NI wavefront instructions per wavefront cover the
// STAGE pieces (instruction c = 4 i + wu moves pieces 64 c .. 64 c + 63);
// addresses past the last piece of S are clamped to it.  ``wu`` is the
// wavefront index in a scalar register.
template <int Q, int STAGE>
__device__ __forceinline__ void wide_stage(const float* S, float* sS, int q0, int sbase, int slast, int wu, int l) {
    int f = (64 * wu + l) / Q, k = (64 * wu + l) - f * Q;
#pragma unroll
    for (int i = 0; i < (STAGE / 64 + 3) / 4; ++i) {
        const int c = 4 * i + wu;
        if (c < STAGE / 64) {
            int src = sbase + f * q0 + k;
            src = src < slast ? src : slast;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const float4*>(S) + src, sS + 4 * 64 * c, 16, 0, 0);
        }
        k += 256 % Q;
        f += 256 / Q;
        if (k >= Q) {
            k -= Q;
            ++f;
        }
    }
}

// Loads of the sample's indices and probability (thread t handles sample
// t % kWideTF of the chunk; clamped), and from them its fiber offset and
// weights in lane order: sample 16 u + r at slot 8 r + u.
struct WideSample {
    int ik[kMaxOrder];
    double pf;
};
__device__ __forceinline__ WideSample wide_sample_load(const int32_t* idx, const double* pF, int f0, int m, int N) {
    WideSample s;
    const int fi = f0 + (threadIdx.x & (kWideTF - 1));
    const int64_t fc = fi < m ? fi : m - 1;
#pragma unroll
    for (int k = 0; k < 3; ++k) s.ik[k] = idx[fc * N + (k < N ? k : N - 1)];
    if (N > 3) {
#pragma unroll
        for (int k = 3; k < kMaxOrder; ++k) s.ik[k] = idx[fc * N + (k < N ? k : N - 1)];
    }
    s.pf = pF[fc];
    return s;
}
__device__ __forceinline__ void wide_sample_meta(const WideSample& s, const tr_desc& d, const WideMode& wm, int n,
                                                 int f0, int m, int64_t* sB, float* sW, double* sL) {
    const int tid = threadIdx.x;
    if (tid >= kWideTF) return;
    bool ok = f0 + tid < m;
    int64_t off = 0;
#pragma unroll
    for (int k = 0; k < kMaxOrder; ++k) {
        if (k >= d.N) break;
        if (k != n && (s.ik[k] < 0 || s.ik[k] >= d.I[k])) ok = false;
        off += (int64_t)s.ik[k] * wm.xs[k];
    }
    const double rp = 1.0 / s.pf;
    const int slot = 8 * (tid & 15) + (tid >> 4);
    sB[slot] = ok ? off : 0;
    sW[slot] = ok ? (float)(wm.wbase * rp) : 0.f;
    sL[slot] = ok ? 0.5 / (double)m * rp : 0.0;
}

}  // namespace trk
