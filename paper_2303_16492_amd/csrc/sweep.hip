// a7/a8 for RR <= 128: the scaled direction p = -g (h + eta I)^{-1}
// (equation eq:scaledsg_direction with the damped preconditioner of the
// remark that follows it), then the step rule.
//
// The RR x RR system is inverted once per step instead of being solved for
// every one of the I_n rows of g: a blocked symmetric sweep (Gauss-Jordan
// elimination on an SPD matrix, eight pivots per block) turns M = h + eta I
// into -M^{-1} in one workgroup, and a second, row-parallel kernel forms
// p = g (-M^{-1}) and applies the rule.  A sweep pivot block is the Schur
// complement of the blocks already swept, so it is positive definite exactly
// when the matching Cholesky pivots are positive: the same test triggers the
// same fallback ladder eta + 10^(k-10) tr(h)/RR, k = 0..6.
//
// The matrix lives in FP64 matrix-core accumulators: 16 x 16 tiles of the
// lower triangle spread over three update wavefronts (tile columns u, 5 - u
// and 6 + u for wavefront u), so each block step moves only the eight pivot
// rows through LDS.  With U~ the pivot columns minus the selector E and
// V~ = U~^T, one block step is the single rank-8 update
//     M <- M - U~ B V~ - 2 E E^T,    B = (M_PP)^{-1},
// which gives -B on the pivot block, B M_PQ on its rows, M_QP B on its
// columns and M_QQ - M_QP B M_PQ elsewhere: the classical sweep.  The
// -2 E E^T term only moves the diagonal of that step's pivot block, which
// no later step reads, so it is applied once at the end.
//
// The fourth wavefront owns no tiles: it works one block ahead.  During
// step q it forms pivot block q+1 as it will be after step q (the Schur
// complement D - C^T B C of the block as published before step q, C the
// pivot rows of step q at its columns, on the vector units) and sweeps that
// 8 x 8 block in registers, so the pivot inverse of every step after the
// first is ready when the step starts.  One barrier per step publishes the next pivot
// rows, the next pivot inverse and its verdict together.
#include "internal.hpp"

namespace trk {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kSweepWaves = 4;
constexpr int kFactorWave = 3;

// Tile columns of update wavefront u = 0, 1, 2: u, 5 - u and 6 + u (those
// below NT).  Slot k of a wavefront walks its columns top to bottom, the
// diagonal tile first; every coordinate is a compile-time constant.
__host__ __device__ constexpr int col_of(int wv, int m) {
    return wv >= kFactorWave ? 99 : (m == 0 ? wv : (m == 1 ? 5 - wv : 6 + wv));
}
template <int NT>
__host__ __device__ constexpr int ncol(int wv, int m) { return NT - col_of(wv, m) > 0 ? NT - col_of(wv, m) : 0; }
template <int NT>
__host__ __device__ constexpr int tiles_of(int wv) { return ncol<NT>(wv, 0) + ncol<NT>(wv, 1) + ncol<NT>(wv, 2); }
template <int NT>
__host__ __device__ constexpr int tpw() {
    int m = 1;
    for (int w = 0; w < kSweepWaves; ++w) m = tiles_of<NT>(w) > m ? tiles_of<NT>(w) : m;
    return m;
}
// which of the wavefront's columns slot k is in (0, 1, 2), or 3 for none
template <int NT>
__host__ __device__ constexpr int s_m(int wv, int k) {
    return k < ncol<NT>(wv, 0) ? 0
                               : (k < ncol<NT>(wv, 0) + ncol<NT>(wv, 1) ? 1 : (k < tiles_of<NT>(wv) ? 2 : 3));
}
template <int NT>
__host__ __device__ constexpr bool s_ok(int wv, int k) { return s_m<NT>(wv, k) < 3; }
template <int NT>
__host__ __device__ constexpr int s_first(int wv, int m) {
    return m == 0 ? 0 : (m == 1 ? ncol<NT>(wv, 0) : ncol<NT>(wv, 0) + ncol<NT>(wv, 1));
}
template <int NT>
__host__ __device__ constexpr int s_ct(int wv, int k) { return s_ok<NT>(wv, k) ? col_of(wv, s_m<NT>(wv, k)) : 0; }
template <int NT>
__host__ __device__ constexpr int s_rt(int wv, int k) {
    return s_ok<NT>(wv, k) ? col_of(wv, s_m<NT>(wv, k)) + k - s_first<NT>(wv, s_m<NT>(wv, k)) : 0;
}

__device__ __forceinline__ int tri8(int i) { return (i * (i + 1)) >> 1; }

// Row pitch (in doubles) of the published pivot rows Vt: 16 NT columns and
// kVtPad more, so that rows u and u + 1 start in different LDS banks (the
// transposed stores of publish_rows and the row reads of the updates touch
// several rows in one instruction; with a pitch of 16 NT doubles, a multiple
// of 32 banks, they all fall in one bank).  At RR = 100 the 13 block steps
// take 38.6 K cycles instead of 40.6 K (paddings of 1, 4 and 8 measured
// within 2% of 2).
constexpr int kVtPad = 2;
template <int NT>
__host__ __device__ constexpr int vt_pitch() { return 16 * NT + kVtPad; }

// 1/p in FP64: the hardware estimate refined by two Newton steps
// y <- y + y (1 - p y) (each squares the relative error).
__device__ __forceinline__ double rcp_nr(double p) {
    double y = __builtin_amdgcn_rcp(p);
    double e = __builtin_fma(-p, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-p, y, 1.0);
    return __builtin_fma(y, e, y);
}

// Symmetric sweep of the 8 x 8 SPD block D8 (row-major, both triangles):
// -D8^{-1}, lower triangle packed by rows (tri8(i) + j) into Bw.  Lane
// 8 i + j of the wavefront holds entry (i, j).  Pivot k takes column k
// (c_x = entry (max(x, k), min(x, k)), lower triangle) by lane permutes,
// then every lane updates its own entry:
//     a_ij -= (c_i / a_kk) c_j,  a_ik <- c_i / a_kk,  a_kj <- c_j / a_kk,
//     a_kk <- -1 / a_kk,
// the classical symmetric sweep.  Only lower-triangle entries are read, so
// the lanes of the lower triangle compute exactly the operations of the
// sequential algorithm on that triangle.  The reciprocal of each next pivot
// is formed one pivot ahead (below), off the chain of lane permutes.  False
// on a pivot not above ``tol`` (0: not positive) or not finite; every lane
// reaches the same verdict.
__device__ __forceinline__ double permute_lane(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Pivot K, dk = 1/a_kk arriving from the previous pivot.  The next pivot
// and its reciprocal are formed here from the two entries they depend on
// (read before this pivot's update, with the very operations lane 9(K+1)
// applies to its entry, so the value is the same bit for bit), and the
// reciprocal chain of pivot K+1 runs while this pivot waits for its lane
// permutes.
template <int K>
__device__ __forceinline__ void sweep8_pivot(double& a, double& dk, bool& good, int i, int j, double tol) {
    const double ci = permute_lane(a, i > K ? 8 * i + K : 8 * K + i);
    const double cj = permute_lane(a, j > K ? 8 * j + K : 8 * K + j);
    double pn = 0.0, dkn = 0.0;
    if (K < 7) {
        const double c1 = readlane_f64(a, 8 * (K + 1) + K);   // entry (K+1, K)
        const double a11 = readlane_f64(a, 9 * (K + 1));
        pn = __builtin_fma(-(c1 * dk), c1, a11);
        dkn = rcp_nr(pn);
    }
    double ti = ci * dk, tj = cj * dk;
    double up = __builtin_fma(-ti, cj, a);
    double nd = -dk;
    asm volatile("" : "+v"(ti), "+v"(tj), "+v"(up), "+v"(nd));   // all four ready: selects, no branches
    a = (i != K) ? ((j != K) ? up : ti) : ((j != K) ? tj : nd);
    if (K < 7) {
        good = good && (pn > tol) && isfinite(pn);
        dk = dkn;
    }
}

// The sweep of the block whose entry (i, j) lane 8 i + j holds in ``a``.
__device__ __forceinline__ bool sweep8_reg(double a, double* Bw, double tol) {
    const int l = threadIdx.x & 63, i = l >> 3, j = l & 7;
    const double p = readlane_f64(a, 0);
    double dk = rcp_nr(p);
    bool good = (p > tol) && isfinite(p);
    sweep8_pivot<0>(a, dk, good, i, j, tol);
    sweep8_pivot<1>(a, dk, good, i, j, tol);
    sweep8_pivot<2>(a, dk, good, i, j, tol);
    sweep8_pivot<3>(a, dk, good, i, j, tol);
    sweep8_pivot<4>(a, dk, good, i, j, tol);
    sweep8_pivot<5>(a, dk, good, i, j, tol);
    sweep8_pivot<6>(a, dk, good, i, j, tol);
    sweep8_pivot<7>(a, dk, good, i, j, tol);
    if (j <= i) Bw[tri8(i) + j] = a;
    return good;
}

__device__ __forceinline__ bool sweep8(const double* __restrict__ D8, double* Bw, double tol) {
    const int l = threadIdx.x & 63;
    return sweep8_reg(D8[(l >> 3) * 8 + (l & 7)], Bw, tol);
}

// Pivot rows of block q = 2 tq + HQ of the current matrix, minus the
// selector, into Vt[u][c] = M(8q + u, c) - [c == 8q + u] for every column
// c < 16 NT (row pitch vt_pitch).  Rows of the pivot tile row come from the tiles left of the
// diagonal; entries right of it from the column of tiles below (M is
// symmetric).  The half HQ of the tile is a compile-time constant, so every
// register index is static; only the tile-row tests (uniform) branch.
template <int NT, int WV, int HQ>
__device__ __forceinline__ void publish_rows(const dbl4 (&acc)[tpw<NT>()], int q, double* Vt) {
    constexpr int NP = vt_pitch<NT>();
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    const int tq = q >> 1;
#pragma unroll
    for (int k = 0; k < tpw<NT>(); ++k) {
        if (!s_ok<NT>(WV, k)) continue;
        const int rt = s_rt<NT>(WV, k), ct = s_ct<NT>(WV, k);
        if (rt == tq) {
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) {
                const double v = acc[k][2 * HQ + jj];
                const int u = 4 * jj + lr, c = 16 * ct + lc;
                // the selector lies in the diagonal tile only: c == 8q + u there is lc == 8 HQ + u
                Vt[u * NP + c] = ct == tq ? v - (lc == 8 * HQ + u ? 1.0 : 0.0) : v;
            }
        } else if (ct == tq && rt > tq && (lc >> 3) == HQ) {
            const int u = lc - 8 * HQ;
#pragma unroll
            for (int j = 0; j < 4; ++j) Vt[u * NP + 16 * rt + 4 * j + lr] = acc[k][j];
        }
    }
}

// The 8 x 8 pivot block 2 t + HQ (plain M_PP, row-major) from its diagonal
// tile t.
template <int HQ>
__device__ __forceinline__ void publish_d8(const dbl4& a, double* D8) {
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    if ((lc >> 3) == HQ) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) D8[(4 * jj + lr) * 8 + (lc - 8 * HQ)] = a[2 * HQ + jj];
    }
}

struct SweepZ {
    dbl4 z[3];
};

// Z = B V~ for the wavefront's tile columns (rows 8..15 of each product are
// zero), with B = M_PP^{-1} = -(packed Bw).
template <int NT, int WV>
__device__ __forceinline__ SweepZ compute_z(const double* __restrict__ Vt, const double* __restrict__ Bw) {
    constexpr int NP = vt_pitch<NT>();
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    double a1[2], v[3][2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int j = 4 * s + lr;
        const int hi = j > lc ? j : lc, lo = j > lc ? lc : j;
        a1[s] = lc < 8 ? -Bw[tri8(hi & 7) + (lo & 7)] : 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][s] = ncol<NT>(WV, m) > 0 ? Vt[j * NP + 16 * col_of(WV, m) + lc] : 0.0;
    }
    const dbl4 zero = {0.0, 0.0, 0.0, 0.0};
    SweepZ z{{zero, zero, zero}};
#pragma unroll
    for (int m = 0; m < 3; ++m)
        if (ncol<NT>(WV, m) > 0) z.z[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[0], v[m][0], zero, 0, 0, 0);
#pragma unroll
    for (int m = 0; m < 3; ++m)
        if (ncol<NT>(WV, m) > 0) z.z[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[1], v[m][1], z.z[m], 0, 0, 0);
    return z;
}

// a - U~ Z on the tile in tile row rt.
template <int NT>
__device__ __forceinline__ dbl4 update_tile(const dbl4& a, const double* __restrict__ Vt, const dbl4& zz, int rt) {
    constexpr int NP = vt_pitch<NT>();
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    double ua[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) ua[s] = -Vt[(4 * s + lr) * NP + 16 * rt + lc];
    const dbl4 r = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[0], zz[0], a, 0, 0, 0);
    return __builtin_amdgcn_mfma_f64_16x16x4f64(ua[1], zz[1], r, 0, 0, 0);
}

// Pivot block q+1 after step q from the block D as published before step q:
// Dn = D - C^T B C with C the pivot rows of step q at the block's columns
// (Schur complement), on the vector units, entry (i, j) in lane 8 i + j (the
// layout of sweep8_reg): w = B C (lane (i, j): row i of B, column j of C),
// exchanged through ``Wt`` (64 doubles of the factor wavefront's own), then
// (C^T w)(i, j) from column i of C and column j of w.  Two dependent 8-term
// products, and the block goes straight into the sweep's registers.
template <int NT>
__device__ __forceinline__ double next_pivot_entry(const double* __restrict__ Vt, const double* __restrict__ Bw,
                                                   const double* __restrict__ D, int q, double* Wt) {
    constexpr int NP = vt_pitch<NT>();
    const int l = threadIdx.x & 63, i = l >> 3, j = l & 7;
    const int c0 = 8 * (q + 1);
    double b[8], c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        b[k] = -Bw[tri8(i > k ? i : k) + (i > k ? k : i)];
        c[k] = Vt[k * NP + c0 + j];
    }
    const double dv = D[i * 8 + j];
    double w0 = 0.0, w1 = 0.0;
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        w0 = __builtin_fma(b[k], c[k], w0);
        w1 = __builtin_fma(b[k + 1], c[k + 1], w1);
    }
    Wt[l] = w0 + w1;
    // this wavefront's LDS stores complete before its own reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double ci[8], wk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        ci[k] = Vt[k * NP + c0 + i];
        wk[k] = Wt[8 * k + j];
    }
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        r0 = __builtin_fma(ci[k], wk[k], r0);
        r1 = __builtin_fma(ci[k + 1], wk[k + 1], r1);
    }
    return dv - (r0 + r1);
}

// h + eta I into the wavefront's tiles (identity on the padding), every
// load issued before any use (indices clamped in bounds, masked after).
template <int NT, int WV>
__device__ __forceinline__ void fill_tiles(dbl4 (&acc)[tpw<NT>()], const double* __restrict__ gram, int RR,
                                           double eta) {
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    double g[tpw<NT>()][4];
#pragma unroll
    for (int k = 0; k < tpw<NT>(); ++k) {
        const int rt = s_rt<NT>(WV, k), ct = s_ct<NT>(WV, k);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 16 * rt + 4 * j + lr, c = 16 * ct + lc;
            const int rc = r < RR ? r : RR - 1, cc = c < RR ? c : RR - 1;
            g[k][j] = s_ok<NT>(WV, k) ? gram[(int64_t)rc * RR + cc] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < tpw<NT>(); ++k) {
        const int rt = s_rt<NT>(WV, k), ct = s_ct<NT>(WV, k);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 16 * rt + 4 * j + lr, c = 16 * ct + lc;
            const bool in = r < RR && c < RR;
            acc[k][j] = (in ? g[k][j] : 0.0) + (r == c ? (r < RR ? eta : 1.0) : 0.0);
        }
    }
}

// -M^{-1} into hm (both triangles), with the deferred -2 on the diagonal,
// scaled back by sc (the sweep ran on sc M).
template <int NT, int WV>
__device__ __forceinline__ void store_tiles(const dbl4 (&acc)[tpw<NT>()], double* __restrict__ hm, int RR,
                                            double sc) {
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
#pragma unroll
    for (int k = 0; k < tpw<NT>(); ++k) {
        if (!s_ok<NT>(WV, k)) continue;
        const int rt = s_rt<NT>(WV, k), ct = s_ct<NT>(WV, k);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 16 * rt + 4 * j + lr, c = 16 * ct + lc;
            if (r < RR && c < RR) {
                hm[(int64_t)r * RR + c] = (acc[k][j] - (r == c ? 2.0 : 0.0)) * sc;
                if (rt != ct) hm[(int64_t)c * RR + r] = acc[k][j] * sc;
            }
        }
    }
}

struct SweepShared {
    double Vt[2][8 * (128 + kVtPad)];   // pivot rows of step q, by q & 1 (pitch vt_pitch)
    double Bw[2][40];        // packed -B of step q, by q & 1
    double D8[2][64];        // pivot block q+1 as published before step q, by (q + 1) & 1
    double Dn[64];           // factor wavefront: pivot block 0 in the prologue, then the exchange of w = B C
    double red[kSweepWaves];
    double mxdiag;           // largest diagonal entry of h, found by the factor wavefront
    int good[2];             // verdict of the factorisation of step q's pivot block, by q & 1
};

// Block step q of one wavefront, ending at the step's barrier; HQ = q & 1
// is a compile-time constant (the half of a tile that holds the pivot rows,
// and the parity of the double-buffered shared arrays).  Update wavefronts
// apply the step to their tiles and publish the next pivot rows; the factor
// wavefront forms pivot block q+1 as it will be after step q and sweeps it.
// Returns the verdict on pivot block q + 1 (true after the last step).
template <int NT, int WV, int HQ>
__device__ __forceinline__ bool sweep_step(dbl4 (&acc)[tpw<NT>()], SweepShared& sh, int q, int npiv, double tol) {
    const double* Vt = sh.Vt[HQ];
    const bool more = q + 1 < npiv;
    if (WV == kFactorWave) {
        if (more) {
            const double a = next_pivot_entry<NT>(Vt, sh.Bw[HQ], sh.D8[HQ ^ 1], q, sh.Dn);
            const bool g = sweep8_reg(a, sh.Bw[HQ ^ 1], tol);
            if ((threadIdx.x & 63) == 0) sh.good[HQ ^ 1] = g ? 1 : 0;
        }
    } else {
        const SweepZ z = compute_z<NT, WV>(Vt, sh.Bw[HQ]);
#pragma unroll
        for (int k = 0; k < tpw<NT>(); ++k)
            if (s_ok<NT>(WV, k)) acc[k] = update_tile<NT>(acc[k], Vt, z.z[s_m<NT>(WV, k)], s_rt<NT>(WV, k));
        if (more) publish_rows<NT, WV, HQ ^ 1>(acc, q + 1, sh.Vt[HQ ^ 1]);
        if (q + 2 < npiv) {
            // pivot block q+2 (same parity) as it stands after this step
            const int t2 = (q + 2) >> 1;
#pragma unroll
            for (int m = 0; m < 3; ++m)
                if (ncol<NT>(WV, m) > 0 && t2 == col_of(WV, m)) publish_d8<HQ>(acc[s_first<NT>(WV, m)], sh.D8[HQ]);
        }
    }
    __syncthreads();
    return more ? sh.good[HQ ^ 1] != 0 : true;
}

// One wavefront's part of the sweep with the fallback ladder.  Returns the
// attempt that succeeded, or -1.  Every wavefront passes the same barriers
// and reads the same verdicts, so every wavefront returns the same value.
// rank_tol > 0: a rank test instead of the ladder; one attempt, and a pivot
// not above rank_tol * max_i h_ii fails it.
//
// The sweep runs on sc (h + eta I) with sc the power of two that puts the
// largest diagonal entry in [0.5, 1) (exact), and the inverse is scaled back
// by sc when stored: the pivot block of every step is held as 2 I - B until
// the deferred -2 I, which keeps B's digits only while B is not far below
// 1, i.e. while the matrix is not far above 1.
template <int NT, int WV>
__device__ __forceinline__ int sweep_wave(const double* __restrict__ gram, int RR, double damping, double rank_tol,
                                          double* __restrict__ hm, SweepShared& sh) {
    const int npiv = (RR + 7) >> 3;
    const int l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    dbl4 acc[tpw<NT>()];
    double base = 0.0;   // tr(h + damping I) / RR, needed only once a factorisation has failed
    double tol = 0.0;
    double sc = 1.0;
    const int attempts = rank_tol > 0.0 ? 1 : 8;
    for (int attempt = 0; attempt < attempts; ++attempt) {
        if (attempt == 1) {
            double tr = 0.0;
            for (int c = threadIdx.x; c < RR; c += blockDim.x) tr += gram[(int64_t)c * RR + c];
            base = (block_sum(tr, sh.red) + damping * RR) / RR;
        }
        const double eta = attempt == 0 ? damping : damping + pow(10.0, (double)(attempt - 1 - 10)) * base;
        // The factor wavefront's loads go out before the barrier below and
        // the update wavefronts' after it, so that the CU serves the first
        // pivot blocks and the diagonal first: the first 8 x 8 sweep then
        // runs while the tiles are still arriving.  Diagonal entries l and
        // l + 64: the factor wavefront alone loads them (64 rows per load;
        // the update wavefronts' loads are their tiles).
        double dg[2] = {0.0, 0.0};
        double xg[2] = {0.0, 0.0};   // factor wavefront: entry (u, v) of pivot blocks 0 and 1 of h
        if (WV == kFactorWave) {
            if (attempt == 0) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int c = l + 64 * u, cc = c < RR ? c : RR - 1;
                    const double v = gram[(int64_t)cc * RR + cc];
                    dg[u] = c < RR ? v : 0.0;
                }
            }
            const int u = l >> 3, v = l & 7;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int r = 8 * b + u, c = 8 * b + v;
                const int rc = r < RR ? r : RR - 1, cc = c < RR ? c : RR - 1;
                xg[b] = gram[(int64_t)rc * RR + cc];
            }
        }
        __syncthreads();   // the previous attempt's readers are done with the shared buffers
        double xb[2];      // factor wavefront: entry (u, v) of pivot blocks 0 and 1 of h + eta I
        if (WV == kFactorWave) {
            const int u = l >> 3, v = l & 7;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int r = 8 * b + u, c = 8 * b + v;
                xb[b] = (r < RR && c < RR ? xg[b] : 0.0) + (r == c ? (r < RR ? eta : 1.0) : 0.0);
            }
        } else {
            fill_tiles<NT, WV>(acc, gram, RR, eta);
        }
        if (attempt == 0) {   // largest diagonal entry of h + eta I, handed out through LDS
            if (WV == kFactorWave) {
                double mx = fmax(dg[0], dg[1]);
                for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
                if (l == 0) sh.mxdiag = mx;
            }
            __syncthreads();
            const double mxa = sh.mxdiag + eta;
            int ex = 0;
            if (mxa > 0.0 && isfinite(mxa)) {
                (void)frexp(mxa, &ex);
                sc = ldexp(1.0, -ex);
            }
            if (rank_tol > 0.0) tol = rank_tol * mxa * sc;
        }
        if (WV == kFactorWave) {
            const int u = l >> 3, v = l & 7;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int r = 8 * b + u, c = 8 * b + v;
                const double x = (r < RR && c < RR) ? xb[b] * sc : xb[b];
                if (b == 0) sh.Dn[u * 8 + v] = x;
                else sh.D8[1][u * 8 + v] = x;
            }
            // this wavefront's LDS stores complete before its own reads
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const bool g = sweep8(sh.Dn, sh.Bw[0], tol);
            if (l == 0) sh.good[0] = g ? 1 : 0;
        } else {
#pragma unroll
            for (int k = 0; k < tpw<NT>(); ++k) {
                const int rt = s_rt<NT>(WV, k), ct = s_ct<NT>(WV, k);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = 16 * rt + 4 * j + lr, c = 16 * ct + lc;
                    acc[k][j] = (r < RR && c < RR) ? acc[k][j] * sc : acc[k][j];
                }
            }
            publish_rows<NT, WV, 0>(acc, 0, sh.Vt[0]);
        }
        __syncthreads();
        // block steps in pairs (even q, then odd q)
        bool good = sh.good[0] != 0;
        for (int q = 0; q < npiv && good; q += 2) {
            good = sweep_step<NT, WV, 0>(acc, sh, q, npiv, tol);
            if (good && q + 1 < npiv) good = sweep_step<NT, WV, 1>(acc, sh, q + 1, npiv, tol);
        }
        if (good) {
            if (WV != kFactorWave) store_tiles<NT, WV>(acc, hm, RR, sc);
            return attempt;
        }
    }
    return -1;
}

// -(gram + eta I)^{-1} into hm (RR x RR, row-major, both triangles), with
// the fallback ladder; flag: 0 ok, 1 damped, 2 failed.  With rank_tol > 0
// (the leverage law) there is no ladder: flag 2 means a pivot at or below
// rank_tol * max_i gram_ii, i.e. the Gram is taken as singular.  256 threads.
template <int NT>
__global__ __launch_bounds__(256) void k_sweep(tr_desc d, ModeSrc ms, const double* __restrict__ gram,
                                               Damp dmp, double rank_tol, double* __restrict__ hm,
                                               int* __restrict__ flag, int32_t* status) {
    uint64_t t;
    int n;
    resolve_mode(ms, d.N, &t, &n);
    const double damping = dmp.at(t);
    const int RR = d.R[n] * d.R[ring_next(n, d.N)];
    __shared__ SweepShared sh;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int ok_at;
    switch (w) {
        case 0: ok_at = sweep_wave<NT, 0>(gram, RR, damping, rank_tol, hm, sh); break;
        case 1: ok_at = sweep_wave<NT, 1>(gram, RR, damping, rank_tol, hm, sh); break;
        case 2: ok_at = sweep_wave<NT, 2>(gram, RR, damping, rank_tol, hm, sh); break;
        default: ok_at = sweep_wave<NT, 3>(gram, RR, damping, rank_tol, hm, sh); break;
    }
    if (threadIdx.x == 0) {
        const int fl = ok_at < 0 ? 2 : (ok_at > 0 ? 1 : 0);
        *flag = fl;
        if (fl == 1) set_status(status, TR_DEV_DAMPED);
        if (fl == 2) set_status(status, TR_DEV_NOT_SPD);
    }
}

constexpr int kApplyRows = 16;
constexpr int kApplyWaves = 4;   // the K range split four ways

// p = g (-M^{-1}), then the rule: one 16 x 16 tile of p per block (rows
// 16 blockIdx.x.., columns 16 blockIdx.y..), so the product spreads over
// as many CUs as there are tiles.  Each of the block's four wavefronts runs
// one chain of FP64 matrix-core steps over its quarter of K (K steps of
// four, K = R_n R_{n+1} <= 128) on its own SIMD; wavefronts 1-3 leave their
// partial tiles in LDS and wavefront 0 adds them in a fixed order and
// applies the rule.  Every operand (the tile's rows of g, its columns of
// -M^{-1}, the core and accumulator entries it updates) is loaded straight
// from global memory with all loads in flight.  With lp.part set, block
// (0, 0) also writes the loss.  With ``step`` set, the block that finishes
// last advances the step counter (after every block has read it).
// SHAPE0: every mode has the same I_n and R_n R_{n+1}, so the loads of g and
// -M^{-1} are issued before the step's mode has arrived.
template <typename TC, bool SHAPE0>
__global__ __launch_bounds__(64 * kApplyWaves) void k_scaled_apply(tr_desc d, ModeSrc ms, const TC* __restrict__ g,
                                                                   LossParts lp, double* __restrict__ loss,
                                                                   const double* __restrict__ hm,
                                                                   const int* __restrict__ flag, MutPtrs cores,
                                                                   MutPtrs accum, tr_step rule, int32_t* status,
                                                                   StepBump step) {
    uint64_t t = 0;
    int n = 0;
    if (!SHAPE0) resolve_mode(ms, d.N, &t, &n);
    const int ns = SHAPE0 ? 0 : n;
    const int In = d.I[ns];
    const int RR = d.R[ns] * d.R[ring_next(ns, d.N)];
    const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ double red[kApplyWaves];
    __shared__ dbl4 part[kApplyWaves - 1][64];
    if (blockIdx.x == 0 && blockIdx.y == 0 && lp.part) {
        const double s = loss_parts_sum(lp, In, red);
        if (threadIdx.x == 0) *loss = s;
    }
    constexpr int KW = 32 / kApplyWaves;            // K steps of 4 per wavefront: RR <= 128
    const int r0 = blockIdx.x * kApplyRows, c = 16 * blockIdx.y + lr;
    const bool live = r0 < In && 16 * (int)blockIdx.y < RR;   // uniform
    const int row = r0 + lr, rowc = row < In ? row : In - 1, cc = c < RR ? c : RR - 1;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    TC* G = nullptr;
    TC* A = nullptr;
    double gold[4] = {0.0, 0.0, 0.0, 0.0}, aold[4] = {0.0, 0.0, 0.0, 0.0};
    int fl = 0;
    if (live) {
        // Loads at clamped (in-bounds) indices, masked afterwards: no load
        // sits behind a branch, so all of them are in flight together (with
        // SHAPE0 the ones that do not need the mode go before its read).
        TC ga[KW];
        double hb[KW];
#pragma unroll
        for (int s = 0; s < KW; ++s) {
            const int ks = w * KW + s, k = 4 * ks + lk, kc = k < RR ? k : RR - 1;
            ga[s] = TC(0);
            hb[s] = 0.0;
            if (4 * ks < RR) {   // uniform
                ga[s] = g[(int64_t)rowc * RR + kc];
                hb[s] = hm[(int64_t)kc * RR + cc];
            }
        }
        TC gv[4], av[4];
        if (w == 0) {   // the entries the rule updates
            fl = *flag;
            if (SHAPE0) resolve_mode(ms, d.N, &t, &n);
            G = static_cast<TC*>(cores.p[n]);
            A = static_cast<TC*>(accum.p[n]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + 4 * j + lk, rc = r < In ? r : In - 1;
                gv[j] = G[(int64_t)rc * RR + cc];
                av[j] = TC(0);
            }
            if (rule.kind == 1) {   // uniform; the accumulator exists only for AdaGrad
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = r0 + 4 * j + lk, rc = r < In ? r : In - 1;
                    av[j] = A[(int64_t)rc * RR + cc];
                }
            }
        }
        double a[KW], b[KW];
#pragma unroll
        for (int s = 0; s < KW; ++s) {
            const int ks = w * KW + s, k = 4 * ks + lk;
            a[s] = (row < In && k < RR) ? (double)ga[s] : 0.0;
            b[s] = (k < RR && c < RR) ? hb[s] : 0.0;
        }
        if (w == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = r0 + 4 * j + lk < In && c < RR;
                gold[j] = in ? (double)gv[j] : 0.0;
                aold[j] = in ? (double)av[j] : 0.0;
            }
        }
#pragma unroll
        for (int s = 0; s < KW; ++s)
            if (4 * (w * KW + s) < RR) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
        if (w > 0) part[w - 1][l] = acc;
    }
    __syncthreads();
    if (live && w == 0) {
#pragma unroll
        for (int v = 0; v < kApplyWaves - 1; ++v) acc += part[v][l];   // fixed order
        if (fl != 2) {   // fl == 2: not positive definite even with damping, core unchanged
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + 4 * j + lk;
                if (r < In && c < RR)
                    apply_rule_loaded<TC>(G, A, (int64_t)r * RR + c, gold[j], aold[j], acc[j], rule, t, status);
            }
        }
    }
    bump_if_last(step, rule.kind == 2);
}

bool sweep_supported(const tr_desc& d) { return shape_of(d).maxRR <= 128; }

hipError_t launch_sweep_inverse(const tr_desc& d, ModeSrc ms, const double* gram, Damp damping, const UpdWs& L,
                                void* ws, int32_t* status, hipStream_t st, double rank_tol) {
    const Shape sh = shape_of(d);
    if (sh.maxRR > 128) return hipErrorInvalidValue;
    char* w = static_cast<char*>(ws);
    double* hm = reinterpret_cast<double*>(w + L.L_off);
    int* flag = reinterpret_cast<int*>(w + L.flag_off);
    const int nt = (sh.maxRR + 15) / 16;
    // The workgroup also reserves the rest of the CU's LDS, which no other
    // workgroup can then share: the sweep is one dependency chain, and
    // waves of a concurrent kernel (the gradient, on the other stream) on
    // its SIMDs would stretch every link of it.
    constexpr size_t kCuLds = 160 * 1024;
    const size_t reserve = (kCuLds - sizeof(SweepShared)) & ~(size_t)1023;
#define TRK_SWEEP(NTV)                                                                                          \
    do {                                                                                                        \
        const size_t dyn = allow_lds(reinterpret_cast<const void*>(&k_sweep<NTV>), reserve) ? reserve : 0;     \
        launch_timed(k_sweep<NTV>, dim3(1), dim3(256), dyn, st, d, ms, gram, damping, rank_tol, hm, flag,   \
                     status);                                                                         \
    } while (0)
    switch (nt) {
        case 1: TRK_SWEEP(1); break;
        case 2: TRK_SWEEP(2); break;
        case 3: TRK_SWEEP(3); break;
        case 4: TRK_SWEEP(4); break;
        case 5: TRK_SWEEP(5); break;
        case 6: TRK_SWEEP(6); break;
        case 7: TRK_SWEEP(7); break;
        default: TRK_SWEEP(8); break;
    }
#undef TRK_SWEEP
    return hipGetLastError();
}

hipError_t launch_sweep_apply(const tr_desc& d, ModeSrc ms, const void* g, LossParts lp, double* loss, MutPtrs cores,
                              MutPtrs accum, tr_step rule, int32_t* status, void* ws, const UpdWs& L, StepBump step,
                              hipStream_t st) {
    const Shape sh = shape_of(d);
    if (sh.maxRR > 128) return hipErrorInvalidValue;
    char* w = static_cast<char*>(ws);
    const double* hm = reinterpret_cast<const double*>(w + L.L_off);
    const int* flag = reinterpret_cast<const int*>(w + L.flag_off);
    const dim3 grid((sh.maxI + kApplyRows - 1) / kApplyRows, (sh.maxRR + 15) / 16);
    bool same = true;
    for (int k = 1; k < d.N; ++k)
        same = same && d.I[k] == d.I[0] && d.R[k] * d.R[(k + 1) % d.N] == d.R[0] * d.R[1 % d.N];
#define TRK_APPLY(TC, S0)                                                                                   \
    hipLaunchKernelGGL((k_scaled_apply<TC, S0>), grid, dim3(64 * kApplyWaves), 0, st, d, ms, static_cast<const TC*>(g), lp, \
                       loss, hm, flag, cores, accum, rule, status, step)
    if (d.core_dtype == TR_F64) {
        if (same) TRK_APPLY(double, true);
        else TRK_APPLY(double, false);
    } else {
        if (same) TRK_APPLY(float, true);
        else TRK_APPLY(float, false);
    }
#undef TRK_APPLY
    return hipGetLastError();
}

hipError_t launch_sweep_update(const tr_desc& d, ModeSrc ms, const double* gram, Damp damping, const void* g,
                               double* loss, MutPtrs cores, MutPtrs accum, tr_step rule, int32_t* status, void* ws,
                               const UpdWs& L, StepBump step, hipStream_t st) {
    hipError_t e = launch_sweep_inverse(d, ms, gram, damping, L, ws, status, st);
    if (e != hipSuccess) return e;
    return launch_sweep_apply(d, ms, g, LossParts{}, loss, cores, accum, rule, status, ws, L, step, st);
}

}  // namespace trk
