// C ABI of include/tr.h: host validation, workspace sizing, dispatch, and
// the multi-step driver (Algorithm TR-BRSGD / TR-ScaledBRSGD).
#include <cstring>
#include <mutex>

#include "internal.hpp"

// Device scratch of tr_run_noalloc, for callers that cannot allocate: one
// copy per GPU the library runs on, held until the process ends.  In host
// code ``scratch`` is only a stand-in for the symbol; its device address on
// the current GPU comes from hipGetSymbolAddress (see noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[TR_NOALLOC_SCRATCH_BYTES];

namespace trk {

Shape shape_of(const tr_desc& d) {
    Shape s;
    for (int k = 0; k < d.N; ++k) {
        const int rr = d.R[k] * d.R[ring_next(k, d.N)];
        if (d.I[k] > s.maxI) s.maxI = d.I[k];
        if (d.R[k] > s.maxR) s.maxR = d.R[k];
        if (rr > s.maxRR) s.maxRR = rr;
        const int64_t J = J_of(d, k);
        if (J > s.maxJ) s.maxJ = J;
    }
    return s;
}

int dtype_size(int dt) {
    switch (dt) {
        case TR_F64: return 8;
        case TR_F32: return 4;
        case TR_F16:
        case TR_BF16: return 2;
        default: return 0;
    }
}

tr_status validate_desc(const tr_desc* d) {
    if (!d) return TR_E_ARG;
    if (d->N < 2 || d->N > kMaxOrder) return TR_E_SHAPE;
    __int128 total = 1;
    for (int k = 0; k < d->N; ++k) {
        if (d->I[k] < 1 || d->R[k] < 1 || d->R[k] > kMaxRank) return TR_E_SHAPE;
        total *= d->I[k];
        if (total > ((__int128)1 << 46)) return TR_E_SHAPE;   // J_n and offsets stay far inside int64
        if (d->x_stride[k] < 0) return TR_E_SHAPE;
    }
    if (d->core_dtype == TR_F64) {
        if (d->x_dtype != TR_F64) return TR_E_DTYPE;
    } else if (d->core_dtype == TR_F32) {
        if (d->x_dtype != TR_F32 && d->x_dtype != TR_F16 && d->x_dtype != TR_BF16) return TR_E_DTYPE;
    } else {
        return TR_E_DTYPE;
    }
    return TR_OK;
}

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static tr_status hip_status(hipError_t e) { return e == hipSuccess ? TR_OK : TR_E_HIP; }

static Ptrs to_ptrs(const void* const* cores, int N) {
    Ptrs p{};
    for (int k = 0; k < N; ++k) p.p[k] = cores[k];
    return p;
}

static tr_status check_cores(const tr_desc* d, const void* const* cores) {
    if (!cores) return TR_E_ARG;
    const size_t es = dtype_size(d->core_dtype);
    for (int k = 0; k < d->N; ++k) {
        if (!cores[k]) return TR_E_ARG;
        if (!aligned(cores[k], es)) return TR_E_ALIGN;
    }
    return TR_OK;
}

__global__ void k_bump(uint64_t* t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *t += 1;
}

hipError_t launch_bump(uint64_t* t_dev, hipStream_t st) {
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, st, t_dev);
    return hipGetLastError();
}

// A kernel, not hipMemsetAsync: tr_run may be captured into a graph.
__global__ void k_zero_u32(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

constexpr int kMaxM = 1 << 24;

// Workspace plan of tr_run.
struct RunWs {
    size_t idx, pF, S, g, gram, idxH, pH, SH, grad, gramws, upd, dist, opt, loss, ctr, mode, total;
    GradWs gl;
    GramWs ml, mlH;
    UpdWs ul;
};

static RunWs run_layout(const tr_problem* p, const tr_config* c) {
    RunWs L{};
    const tr_desc& d = p->desc;
    const Shape sh = shape_of(d);
    const size_t es = dtype_size(d.core_dtype);
    const int m = c->m, mH = c->m_H;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes ? bytes : 1);
        return at;
    };
    L.idx = take((size_t)m * d.N * 4);
    L.pF = take((size_t)m * 8);
    L.S = take((size_t)m * sh.maxRR * es);
    L.g = take((size_t)sh.maxI * sh.maxRR * es);
    L.gram = take((size_t)sh.maxRR * sh.maxRR * 8);
    L.idxH = take(mH > 0 ? (size_t)mH * d.N * 4 : 0);
    L.pH = take(mH > 0 ? (size_t)mH * 8 : 0);
    L.SH = take(mH > 0 ? (size_t)mH * sh.maxRR * es : 0);
    L.gl = grad_ws_layout(d, m, c->prec);
    L.grad = take(L.gl.total);
    L.ml = gram_ws_layout(d, m);
    L.mlH = gram_ws_layout(d, mH > 0 ? mH : m);
    L.gramws = take(L.ml.total > L.mlH.total ? L.ml.total : L.mlH.total);
    L.ul = upd_ws_layout(d);
    L.upd = take(L.ul.total);
    L.dist = take(dist_ws_bytes(d, c->law));
    L.opt = take(c->law == TR_LAW_OPTIMAL ? dist_opt_ws_bytes(d) : 0);
    L.loss = take(8);
    L.ctr = take(4);
    L.mode = take(4);
    L.total = o;
    return L;
}

// Workspace of tr_sweep_run: the step driver's layout for the largest block
// (every column J_n for the full-batch methods, m for TR-ALS-Sampled), then
// a copy of every core (the iterate a TR-GD / TR-ScaledGD sweep starts from).
struct SweepRunWs {
    RunWs r;
    size_t snap, total;
    size_t snap_off[kMaxOrder];
};

static bool sweep_full(int method) { return method == TR_METHOD_GD || method == TR_METHOD_SCALED_GD || method == TR_METHOD_ALS; }

static tr_config sweep_as_config(const tr_problem* p, const tr_sweep_config* c) {
    tr_config r{};
    r.m = sweep_full(c->method) ? (int)shape_of(p->desc).maxJ : c->m;
    r.m_H = 0;
    r.law = sweep_full(c->method) ? TR_LAW_UNIFORM : c->law;
    r.scaled = c->method != TR_METHOD_GD;
    r.prec = c->prec;
    r.damping = c->damping;
    r.seed = c->seed;
    return r;
}

static SweepRunWs sweep_layout(const tr_problem* p, const tr_sweep_config* c) {
    SweepRunWs L{};
    const tr_config rc = sweep_as_config(p, c);
    L.r = run_layout(p, &rc);
    const tr_desc& d = p->desc;
    const size_t es = dtype_size(d.core_dtype);
    size_t o = L.r.total;
    L.snap = o;
    for (int k = 0; k < d.N; ++k) {
        L.snap_off[k] = o;
        o += align_up((size_t)d.I[k] * d.R[k] * d.R[ring_next(k, d.N)] * es);
    }
    L.total = o;
    return L;
}

}  // namespace trk

using namespace trk;

extern "C" {

int32_t tr_abi_version(void) { return TR_ABI_VERSION; }

const char* tr_status_str(int32_t s) {
    switch (s) {
        case TR_OK: return "ok";
        case TR_E_ARG: return "invalid argument (null pointer or bad scalar)";
        case TR_E_SHAPE: return "unsupported shape (order, size, rank or batch out of range)";
        case TR_E_DTYPE: return "unsupported dtype combination";
        case TR_E_ALIGN: return "pointer not aligned to its element size";
        case TR_E_WORKSPACE: return "workspace too small";
        case TR_E_HIP: return "HIP runtime or launch error";
        case TR_E_UNSUPPORTED: return "request not supported by this library";
        default: return "unknown status";
    }
}

int32_t tr_mode(uint64_t seed, uint64_t step, int32_t N) {
    if (N < 1) return -1;
    return pick_mode(seed, step, N);
}

size_t tr_dist_workspace_size(const tr_desc* d, int32_t k, int32_t law) {
    if (validate_desc(d) != TR_OK) return 0;
    (void)k;
    return dist_ws_bytes(*d, law);
}

tr_status tr_dist(const tr_desc* d, int32_t k, int32_t law, const void* core_k, uint64_t* cdf_k,
                  int32_t* dev_status, void* ws, size_t ws_bytes, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (k < 0 || k >= d->N || !core_k || !cdf_k) return TR_E_ARG;
    if (law != TR_LAW_LEVERAGE && law != TR_LAW_EUCLID) return TR_E_ARG;
    if (ws_bytes < dist_ws_bytes(*d, law) || !ws) return TR_E_WORKSPACE;
    Ptrs cores{};
    cores.p[k] = core_k;
    uint64_t* outs[kMaxOrder] = {};
    outs[k] = cdf_k;
    ModeSrc ms{nullptr, 0, k, 0};
    return hip_status(launch_dist(*d, ms, false, k, law, cores, outs, dev_status, ws, (hipStream_t)stream));
}

size_t tr_dist_optimal_workspace_size(const tr_desc* d, int32_t n) {
    if (validate_desc(d) != TR_OK) return 0;
    (void)n;
    return dist_opt_ws_bytes(*d);
}

tr_status tr_dist_optimal(const tr_desc* d, int32_t n, const void* const* cores, const void* X, uint64_t* cdf_J,
                          int32_t* dev_status, void* ws, size_t ws_bytes, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if ((s = check_cores(d, cores)) != TR_OK) return s;
    if (n < 0 || n >= d->N || !X || !cdf_J) return TR_E_ARG;
    if (!ws || ws_bytes < dist_opt_ws_bytes(*d)) return TR_E_WORKSPACE;
    XSrc xs{};
    xs.X = X;
    ModeSrc ms{nullptr, 0, n, 0};
    return hip_status(launch_dist_optimal(*d, ms, to_ptrs(cores, d->N), xs, cdf_J, dev_status, ws,
                                          (hipStream_t)stream));
}

tr_status tr_sample(const tr_desc* d, uint64_t seed, uint64_t step, int32_t n, int32_t m,
                    const uint64_t* const* cdf, const uint64_t* cdf_J, int32_t stream_tag, int32_t* idx,
                    double* pF, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (n < 0 || n >= d->N) return TR_E_ARG;
    if (m < 0 || m > kMaxM) return TR_E_SHAPE;
    if (m == 0) return TR_OK;
    if (!idx || !pF) return TR_E_ARG;
    if (!aligned(idx, 4) || !aligned(pF, 8)) return TR_E_ALIGN;
    if (stream_tag < 0) return TR_E_ARG;
    CdfPtrs c{};
    if (cdf && !cdf_J)
        for (int k = 0; k < d->N; ++k) c.p[k] = k == n ? nullptr : cdf[k];
    ModeSrc ms{nullptr, step, n, seed};
    return hip_status(launch_sample_subchain(*d, ms, m, c, cdf_J, stream_tag, Ptrs{}, idx, pF, nullptr, true,
                                             false, (hipStream_t)stream));
}

tr_status tr_subchain(const tr_desc* d, int32_t n, const void* const* cores, const int32_t* idx, int32_t m, void* S,
                      tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (n < 0 || n >= d->N) return TR_E_ARG;
    if (m < 0 || m > kMaxM) return TR_E_SHAPE;
    if (m == 0) return TR_OK;
    if ((s = check_cores(d, cores)) != TR_OK) return s;
    if (!idx || !S) return TR_E_ARG;
    if (!aligned(S, dtype_size(d->core_dtype))) return TR_E_ALIGN;
    ModeSrc ms{nullptr, 0, n, 0};
    return hip_status(launch_sample_subchain(*d, ms, m, CdfPtrs{}, nullptr, 0, to_ptrs(cores, d->N),
                                             const_cast<int32_t*>(idx), nullptr, S, false, true,
                                             (hipStream_t)stream));
}

static tr_status check_prec(const tr_desc* d, int32_t prec) {
    if (d->core_dtype == TR_F64) return prec == TR_PREC_F64 ? TR_OK : TR_E_DTYPE;
    if (d->x_dtype == TR_BF16) return TR_E_UNSUPPORTED;
    if (prec == TR_PREC_F32 || prec == TR_PREC_BF16 || prec == TR_PREC_F16) return TR_OK;
    return TR_E_DTYPE;
}

size_t tr_grad_workspace_size(const tr_desc* d, int32_t m, int32_t prec) {
    if (validate_desc(d) != TR_OK || m <= 0) return 0;
    const GradWs L = grad_ws_layout(*d, m, prec);
    const GramWs M = gram_ws_layout(*d, m);
    return L.total > M.total ? L.total : M.total;
}

tr_status tr_grad(const tr_desc* d, int32_t n, const void* core_n, const void* X, const int32_t* idx, const void* S,
                  const double* pF, int32_t m, int32_t prec, void* g, double* loss, double* gram, void* ws,
                  size_t ws_bytes, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (n < 0 || n >= d->N) return TR_E_ARG;
    if (m < 1 || m > kMaxM) return TR_E_SHAPE;
    if (!core_n || !X || !idx || !S || !pF || !g) return TR_E_ARG;
    if ((s = check_prec(d, prec)) != TR_OK) return s;
    if (!ws || ws_bytes < tr_grad_workspace_size(d, m, prec)) return TR_E_WORKSPACE;
    if (!aligned(ws, 256)) return TR_E_ALIGN;
    hipStream_t st = (hipStream_t)stream;
    Ptrs cores{};
    cores.p[n] = core_n;
    XSrc xs{};
    xs.X = X;
    ModeSrc ms{nullptr, 0, n, 0};
    const GradWs L = grad_ws_layout(*d, m, prec);
    hipError_t e = launch_grad_partial(*d, ms, cores, xs, idx, S, pF, m, prec, ws, L, st);
    if (e == hipSuccess)
        e = launch_grad_reduce(*d, ms, ws, L, g, loss, false, MutPtrs{}, MutPtrs{}, tr_step{}, nullptr, st);
    if (e == hipSuccess && gram) e = launch_gram(*d, ms, S, pF, m, gram, ws, gram_ws_layout(*d, m), st);
    return hip_status(e);
}

size_t tr_gram_workspace_size(const tr_desc* d, int32_t m_H) {
    if (validate_desc(d) != TR_OK || m_H <= 0) return 0;
    return gram_ws_layout(*d, m_H).total;
}

tr_status tr_gram(const tr_desc* d, int32_t n, const void* S_H, const double* pH, int32_t m_H, double* gram,
                  void* ws, size_t ws_bytes, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (n < 0 || n >= d->N) return TR_E_ARG;
    if (m_H < 1 || m_H > kMaxM) return TR_E_SHAPE;
    if (!S_H || !pH || !gram) return TR_E_ARG;
    const GramWs L = gram_ws_layout(*d, m_H);
    if (!ws || ws_bytes < L.total) return TR_E_WORKSPACE;
    ModeSrc ms{nullptr, 0, n, 0};
    return hip_status(launch_gram(*d, ms, S_H, pH, m_H, gram, ws, L, (hipStream_t)stream));
}

size_t tr_update_workspace_size(const tr_desc* d, int32_t n, int32_t scaled) {
    if (validate_desc(d) != TR_OK) return 0;
    (void)n;
    return scaled ? upd_ws_layout(*d).total : 256;
}

tr_status tr_update(const tr_desc* d, int32_t n, void* core_n, const void* g, const double* gram, double damping,
                    const tr_step* rule, uint64_t t, void* accum_n, int32_t* dev_status, void* ws, size_t ws_bytes,
                    tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (n < 0 || n >= d->N || !core_n || !g || !rule) return TR_E_ARG;
    if (rule->kind < 0 || rule->kind > 2) return TR_E_ARG;
    if (rule->kind == 1 && !accum_n) return TR_E_ARG;
    if (rule->kind == 2 && !(rule->tau > 0.0)) return TR_E_ARG;
    if (!(damping >= 0.0)) return TR_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    MutPtrs cores{}, acc{};
    cores.p[n] = core_n;
    acc.p[n] = accum_n;
    ModeSrc ms{nullptr, t, n, 0};
    if (gram) {
        const UpdWs L = upd_ws_layout(*d);
        if (!ws || ws_bytes < L.total) return TR_E_WORKSPACE;
        return hip_status(launch_scaled_update(*d, ms, gram, damping, g, cores, acc, *rule, dev_status, ws, L, st));
    }
    return hip_status(launch_plain_update(*d, ms, g, cores, acc, *rule, dev_status, st));
}

size_t tr_relerr_workspace_size(const tr_desc* d) {
    if (validate_desc(d) != TR_OK) return 0;
    return relerr_ws_bytes(*d);
}

tr_status tr_relerr(const tr_desc* d, const void* const* cores, const void* X_true, double x_true_norm2, double* rse,
                    void* ws, size_t ws_bytes, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if ((s = check_cores(d, cores)) != TR_OK) return s;
    if (!X_true || !rse) return TR_E_ARG;
    if (d->x_dtype == TR_BF16) return TR_E_UNSUPPORTED;
    if (!ws || ws_bytes < relerr_ws_bytes(*d)) return TR_E_WORKSPACE;
    return hip_status(launch_relerr(*d, to_ptrs(cores, d->N), X_true, x_true_norm2, rse, ws, (hipStream_t)stream));
}

tr_status tr_reconstruct(const tr_desc* d, const void* const* cores, void* X, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if ((s = check_cores(d, cores)) != TR_OK) return s;
    if (!X) return TR_E_ARG;
    if (d->x_dtype == TR_BF16) return TR_E_UNSUPPORTED;
    return hip_status(launch_reconstruct(*d, to_ptrs(cores, d->N), X, (hipStream_t)stream));
}

tr_status tr_x_replicate(const tr_desc* d, const void* X, int32_t n, void* Xn, tr_stream_t stream) {
    tr_status s = validate_desc(d);
    if (s != TR_OK) return s;
    if (n < 0 || n >= d->N || !X || !Xn) return TR_E_ARG;
    return hip_status(launch_replicate(*d, X, n, Xn, (hipStream_t)stream));
}

size_t tr_run_workspace_size(const tr_problem* p, const tr_config* c) {
    if (!p || !c || validate_desc(&p->desc) != TR_OK || c->m < 1) return 0;
    return run_layout(p, c).total;
}

tr_status tr_run(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps, double* loss_out,
                 int32_t* dev_status, void* ws, size_t ws_bytes, tr_stream_t stream) {
    return tr_run_ex(p, c, t_dev, steps, loss_out, dev_status, ws, ws_bytes, stream, nullptr);
}

tr_status tr_run_events(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps, double* loss_out,
                        int32_t* dev_status, void* ws, size_t ws_bytes, void* const* ev_begin, void* const* ev_end,
                        tr_stream_t stream) {
    tr_run_opts o{};
    o.ev_begin = ev_begin;
    o.ev_end = ev_end;
    return tr_run_ex(p, c, t_dev, steps, loss_out, dev_status, ws, ws_bytes, stream, &o);
}

tr_status tr_run_ex(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps, double* loss_out,
                    int32_t* dev_status, void* ws, size_t ws_bytes, tr_stream_t stream, const tr_run_opts* opts) {
    const tr_run_opts o = opts ? *opts : tr_run_opts{};
    void* const* ev_begin = o.ev_begin;
    void* const* ev_end = o.ev_end;
    if (!p || !c || !t_dev) return TR_E_ARG;
    const bool any_aux = o.aux || o.ev_fork || o.ev_gram || o.ev_join;
    if (any_aux && !(o.aux && o.ev_fork && o.ev_gram && o.ev_join)) return TR_E_ARG;
    const tr_desc& d = p->desc;
    tr_status s = validate_desc(&d);
    if (s != TR_OK) return s;
    if ((s = check_cores(&d, const_cast<const void* const*>(p->cores))) != TR_OK) return s;
    if (!p->X) return TR_E_ARG;
    if (c->m < 1 || c->m > kMaxM || c->m_H < 0 || c->m_H > kMaxM) return TR_E_SHAPE;
    if (c->law < TR_LAW_UNIFORM || c->law > TR_LAW_OPTIMAL) return TR_E_ARG;
    if ((s = check_prec(&d, c->prec)) != TR_OK) return s;
    if (c->rule.kind < 0 || c->rule.kind > 2) return TR_E_ARG;
    if (c->rule.kind == 2 && !(c->rule.tau > 0.0)) return TR_E_ARG;
    if (!(c->damping >= 0.0)) return TR_E_ARG;
    if (c->damping_schedule < 0 || c->damping_schedule > 2) return TR_E_ARG;
    if (c->damping_schedule == 1 && !(c->damping_tau > 0.0)) return TR_E_ARG;
    if (c->damping_schedule == 2 && !(c->damping_tau > 0.0 && c->damping_tau <= 1.0)) return TR_E_ARG;
    if (c->rule.kind == 1)
        for (int k = 0; k < d.N; ++k)
            if (!p->accum[k]) return TR_E_ARG;
    if (c->law == TR_LAW_LEVERAGE || c->law == TR_LAW_EUCLID)
        for (int k = 0; k < d.N; ++k)
            if (!p->cdf[k]) return TR_E_ARG;
    if (c->law == TR_LAW_OPTIMAL && !p->cdf_J) return TR_E_ARG;
    if (steps < 0) return TR_E_ARG;
    const RunWs L = run_layout(p, c);
    if (!ws || ws_bytes < L.total) return TR_E_WORKSPACE;
    if (!aligned(ws, 256)) return TR_E_ALIGN;
    if (steps == 0) return TR_OK;

    hipStream_t st = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    int32_t* idx = reinterpret_cast<int32_t*>(w + L.idx);
    double* pF = reinterpret_cast<double*>(w + L.pF);
    void* S = w + L.S;
    void* g = w + L.g;
    double* gram = reinterpret_cast<double*>(w + L.gram);
    double* lossw = reinterpret_cast<double*>(w + L.loss);
    Ptrs cores{};
    MutPtrs mcores{}, acc{};
    CdfPtrs cdf{};
    XSrc xs{};
    xs.X = p->X;
    for (int k = 0; k < d.N; ++k) {
        cores.p[k] = p->cores[k];
        mcores.p[k] = p->cores[k];
        acc.p[k] = p->accum[k];
        xs.rep[k] = p->Xrep[k];
        if (c->law == TR_LAW_LEVERAGE || c->law == TR_LAW_EUCLID) cdf.p[k] = p->cdf[k];
    }
    hipError_t e = hipSuccess;
    const bool refresh = c->law == TR_LAW_LEVERAGE || c->law == TR_LAW_EUCLID;
    // The step counter advances in the last kernel of a step: the update,
    // or for E/L the law refresh that reads the step's mode after it.
    unsigned* ctr = reinterpret_cast<unsigned*>(w + L.ctr);
    const StepBump fused = refresh ? StepBump{} : StepBump{t_dev, ctr};
    if (!refresh) e = launch_zero_u32(ctr, 1, st);
    if (refresh)
        for (int k = 0; k < d.N && e == hipSuccess; ++k)
            e = launch_dist(d, ModeSrc{nullptr, 0, k, 0}, false, k, c->law, cores, p->cdf, dev_status,
                            w + L.dist, st);
    // The Gram, its reduction and the inverse use the mode only for R_n R_{n+1}
    // and J_n; when every mode has the same ones they take mode 0 and skip
    // the dependent read of the step counter.
    bool same_shape = true;
    for (int k = 1; k < d.N; ++k)
        same_shape = same_shape && d.R[k] * d.R[(k + 1) % d.N] == d.R[0] * d.R[1 % d.N] && d.I[k] == d.I[0];
    // The step's first kernel draws its mode from (seed, t) and publishes it;
    // the later kernels of the step read it instead of drawing it again.
    int32_t* nslot = reinterpret_cast<int32_t*>(w + L.mode);
    const bool sched = c->damping_schedule != 0;
    const Damp damp(c->damping, c->damping_tau, c->damping_schedule);
    for (int it = 0; it < steps && e == hipSuccess; ++it) {
        const ModeSrc ms_draw{t_dev, 0, -1, c->seed, nullptr, nslot};
        const ModeSrc ms{t_dev, 0, -2, c->seed, nslot, nullptr};
        // a damping schedule needs t: then the shape-only kernels read it too
        const ModeSrc ms_shape = same_shape ? ModeSrc{sched ? t_dev : nullptr, 0, 0, c->seed} : ms;
        double* loss = loss_out ? loss_out + it : lossw;
        // Scaled steps (RR <= 128) with a second stream: the Gram, its
        // reduction and the inverse need only the draws, so they run on
        // ``hs``; the gradient waits for the Gram's group sums (it is not
        // on the critical path) and then runs beside the reduction and the
        // inverse, and the gradient partials are added on ``st`` too.
        // With an independent H draw and modes of one shape, nothing on
        // ``hs`` reads the step's draws: the branch forks before them, and
        // its sample kernel draws the step's mode itself (the same counter,
        // so the same mode) and runs beside the step's own.
        const bool fork = any_aux && c->scaled && sweep_supported(d);
        const bool fork_early = fork && c->m_H > 0 && same_shape;
        hipStream_t hs = fork ? (hipStream_t)o.aux : st;
        if (c->law == TR_LAW_OPTIMAL)
            e = launch_dist_optimal(d, ms_draw, cores, xs, p->cdf_J, dev_status, w + L.opt, st);
        if (e == hipSuccess && fork_early) {
            e = hipEventRecord((hipEvent_t)o.ev_fork, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(hs, (hipEvent_t)o.ev_fork, 0);
        }
        if (e == hipSuccess)
            e = launch_sample_subchain(d, ms_draw, c->m, cdf, c->law == TR_LAW_OPTIMAL ? p->cdf_J : nullptr,
                                       TR_STREAM_IDX, cores, idx, pF, S, true, true, st);
        if (c->scaled && sweep_supported(d)) {
            const Shape sh = shape_of(d);
            if (e == hipSuccess && fork && !fork_early) {
                e = hipEventRecord((hipEvent_t)o.ev_fork, st);
                if (e == hipSuccess) e = hipStreamWaitEvent(hs, (hipEvent_t)o.ev_fork, 0);
            }
            if (e == hipSuccess) {
                if (c->m_H > 0) {
                    int32_t* idxH = reinterpret_cast<int32_t*>(w + L.idxH);
                    double* pH = reinterpret_cast<double*>(w + L.pH);
                    void* SH = w + L.SH;
                    const ModeSrc ms_h = fork_early ? ModeSrc{t_dev, 0, -1, c->seed, nullptr, nullptr} : ms;
                    e = launch_sample_subchain(d, ms_h, c->m_H, cdf, c->law == TR_LAW_OPTIMAL ? p->cdf_J : nullptr,
                                               TR_STREAM_H, cores, idxH, pH, SH, true, true, hs);
                    if (e == hipSuccess)
                        e = launch_gram(d, ms_shape, SH, pH, c->m_H, gram, w + L.gramws, L.mlH, hs,
                                        fork ? (hipEvent_t)o.ev_gram : nullptr);
                } else {
                    e = launch_gram(d, ms_shape, S, pF, c->m, gram, w + L.gramws, L.ml, hs,
                                    fork ? (hipEvent_t)o.ev_gram : nullptr);
                }
            }
            if (e == hipSuccess) {
                TimedDispatch td(o.ev_inv_begin ? (hipEvent_t)o.ev_inv_begin[it] : nullptr,
                                 o.ev_inv_end ? (hipEvent_t)o.ev_inv_end[it] : nullptr);
                e = launch_sweep_inverse(d, ms_shape, gram, damp, L.ul, w + L.upd, dev_status, hs);
            }
            if (e == hipSuccess && fork) e = hipEventRecord((hipEvent_t)o.ev_join, hs);
            if (e == hipSuccess && fork) e = hipStreamWaitEvent(st, (hipEvent_t)o.ev_gram, 0);
            if (e == hipSuccess) {
                TimedDispatch td(ev_begin ? (hipEvent_t)ev_begin[it] : nullptr,
                                 ev_end ? (hipEvent_t)ev_end[it] : nullptr);
                e = launch_grad_partial(d, ms, cores, xs, idx, S, pF, c->m, c->prec, w + L.grad, L.gl, st);
            }
            if (e == hipSuccess)
                e = launch_grad_reduce(d, ms, w + L.grad, L.gl, g, loss, false, MutPtrs{}, MutPtrs{}, c->rule,
                                       dev_status, st);
            if (e == hipSuccess && fork) e = hipStreamWaitEvent(st, (hipEvent_t)o.ev_join, 0);
            if (e == hipSuccess)
                e = launch_sweep_apply(d, ms, g, LossParts{}, nullptr, mcores, acc, c->rule, dev_status, w + L.upd,
                                       L.ul, fused, st);
        } else {
            if (e == hipSuccess) {
                TimedDispatch td(ev_begin ? (hipEvent_t)ev_begin[it] : nullptr,
                                 ev_end ? (hipEvent_t)ev_end[it] : nullptr);
                e = launch_grad_partial(d, ms, cores, xs, idx, S, pF, c->m, c->prec, w + L.grad, L.gl, st);
            }
            if (e != hipSuccess) break;
            if (c->scaled) {   // RR > 128: Cholesky path
                e = launch_grad_reduce(d, ms, w + L.grad, L.gl, g, loss, false, MutPtrs{}, MutPtrs{}, c->rule,
                                       dev_status, st);
                if (e == hipSuccess) {
                    if (c->m_H > 0) {
                        int32_t* idxH = reinterpret_cast<int32_t*>(w + L.idxH);
                        double* pH = reinterpret_cast<double*>(w + L.pH);
                        void* SH = w + L.SH;
                        e = launch_sample_subchain(d, ms, c->m_H, cdf,
                                                   c->law == TR_LAW_OPTIMAL ? p->cdf_J : nullptr, TR_STREAM_H, cores,
                                                   idxH, pH, SH, true, true, st);
                        if (e == hipSuccess) e = launch_gram(d, ms, SH, pH, c->m_H, gram, w + L.gramws, L.mlH, st);
                    } else {
                        e = launch_gram(d, ms, S, pF, c->m, gram, w + L.gramws, L.ml, st);
                    }
                }
                if (e == hipSuccess)
                    e = launch_scaled_update(d, ms, gram, damp, g, mcores, acc, c->rule, dev_status, w + L.upd,
                                             L.ul, st);
                if (e == hipSuccess && fused.t) e = launch_bump(t_dev, st);
            } else {
                e = launch_grad_reduce(d, ms, w + L.grad, L.gl, nullptr, loss, true, mcores, acc, c->rule,
                                       dev_status, st, fused);
            }
        }
        if (e == hipSuccess && refresh)   // the law's last kernel also advances the step counter
            e = launch_dist(d, ms, true, 0, c->law, cores, p->cdf, dev_status, w + L.dist, st, t_dev);
    }
    return hip_status(e);
}

static tr_status check_sweep(const tr_problem* p, const tr_sweep_config* c) {
    if (!p || !c) return TR_E_ARG;
    const tr_desc& d = p->desc;
    tr_status s = validate_desc(&d);
    if (s != TR_OK) return s;
    if ((s = check_cores(&d, const_cast<const void* const*>(p->cores))) != TR_OK) return s;
    if (!p->X) return TR_E_ARG;
    if (c->method < TR_METHOD_GD || c->method > TR_METHOD_ALS_SAMPLED) return TR_E_ARG;
    if ((s = check_prec(&d, c->prec)) != TR_OK) return s;
    if (!(c->damping >= 0.0)) return TR_E_ARG;
    if (sweep_full(c->method)) {
        if (shape_of(d).maxJ > kMaxM) return TR_E_SHAPE;
        if (c->method == TR_METHOD_GD && !(c->alpha > 0.0)) return TR_E_ARG;
        if (c->method == TR_METHOD_SCALED_GD && !(c->alpha > 0.0)) return TR_E_ARG;
    } else {
        if (c->m < 1 || c->m > kMaxM) return TR_E_SHAPE;
        if (c->law != TR_LAW_UNIFORM && c->law != TR_LAW_LEVERAGE && c->law != TR_LAW_EUCLID) return TR_E_UNSUPPORTED;
        if (c->law != TR_LAW_UNIFORM)
            for (int k = 0; k < d.N; ++k)
                if (!p->cdf[k]) return TR_E_ARG;
    }
    return TR_OK;
}

size_t tr_sweep_workspace_size(const tr_problem* p, const tr_sweep_config* c) {
    if (check_sweep(p, c) != TR_OK) return 0;
    return sweep_layout(p, c).total;
}

tr_status tr_sweep_run(const tr_problem* p, const tr_sweep_config* c, uint64_t* t_dev, int32_t sweeps,
                       int32_t* dev_status, void* ws, size_t ws_bytes, tr_stream_t stream) {
    tr_status s = check_sweep(p, c);
    if (s != TR_OK) return s;
    if (!t_dev || sweeps < 0) return TR_E_ARG;
    const SweepRunWs SL = sweep_layout(p, c);
    if (!ws || ws_bytes < SL.total) return TR_E_WORKSPACE;
    if (!aligned(ws, 256)) return TR_E_ALIGN;
    if (sweeps == 0) return TR_OK;
    const RunWs& L = SL.r;
    const tr_desc& d = p->desc;
    const tr_config rc = sweep_as_config(p, c);
    hipStream_t st = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    int32_t* idx = reinterpret_cast<int32_t*>(w + L.idx);
    double* pF = reinterpret_cast<double*>(w + L.pF);
    void* S = w + L.S;
    void* g = w + L.g;
    double* gram = reinterpret_cast<double*>(w + L.gram);
    double* lossw = reinterpret_cast<double*>(w + L.loss);
    const bool full = sweep_full(c->method);
    const bool jacobi = c->method == TR_METHOD_GD || c->method == TR_METHOD_SCALED_GD;
    const bool refresh = !full && (c->law == TR_LAW_LEVERAGE || c->law == TR_LAW_EUCLID);
    const size_t es = dtype_size(d.core_dtype);
    Ptrs live{}, rd{};
    MutPtrs mcores{}, acc{};
    CdfPtrs cdf{};
    XSrc xs{};
    xs.X = p->X;
    for (int k = 0; k < d.N; ++k) {
        live.p[k] = p->cores[k];
        mcores.p[k] = p->cores[k];
        rd.p[k] = jacobi ? static_cast<const void*>(w + SL.snap_off[k]) : p->cores[k];
        xs.rep[k] = p->Xrep[k];
        if (refresh) cdf.p[k] = p->cdf[k];
    }
    hipError_t e = hipSuccess;
    if (refresh)
        for (int k = 0; k < d.N && e == hipSuccess; ++k)
            e = launch_dist(d, ModeSrc{nullptr, 0, k, 0}, false, k, c->law, live, p->cdf, dev_status, w + L.dist, st);
    for (int sw = 0; sw < sweeps && e == hipSuccess; ++sw) {
        if (jacobi)   // the iterate every block of this sweep is computed from
            for (int k = 0; k < d.N && e == hipSuccess; ++k)
                e = hipMemcpyAsync(w + SL.snap_off[k], p->cores[k],
                                   (size_t)d.I[k] * d.R[k] * d.R[ring_next(k, d.N)] * es, hipMemcpyDeviceToDevice, st);
        for (int n = 0; n < d.N && e == hipSuccess; ++n) {
            const ModeSrc ms{t_dev, 0, n, c->seed, nullptr, nullptr};
            const int64_t Jn = J_of(d, n);
            const int m = full ? (int)Jn : c->m;
            e = launch_sample_subchain_mode(d, ms, m, cdf, nullptr, TR_STREAM_IDX, rd, idx, pF, S, full ? 2 : 1, true,
                                            st);
            if (e == hipSuccess) e = launch_grad_partial(d, ms, rd, xs, idx, S, pF, m, c->prec, w + L.grad, L.gl, st);
            if (e != hipSuccess) break;
            if (c->method == TR_METHOD_GD) {
                // g = grad f / J_n over every column: G -= alpha grad f is the
                // rule's fixed step alpha J_n along p = -g
                tr_step rule{};
                rule.kind = 0;
                rule.alpha = c->alpha * (double)Jn;
                e = launch_grad_reduce(d, ms, w + L.grad, L.gl, nullptr, lossw, true, mcores, acc, rule, dev_status,
                                       st);
            } else {
                tr_step rule{};
                rule.kind = 0;
                rule.alpha = c->method == TR_METHOD_SCALED_GD ? c->alpha : 1.0;
                e = launch_grad_reduce(d, ms, w + L.grad, L.gl, g, lossw, false, MutPtrs{}, MutPtrs{}, rule,
                                       dev_status, st);
                if (e == hipSuccess) e = launch_gram(d, ms, S, pF, m, gram, w + L.gramws, L.ml, st);
                if (e == hipSuccess)
                    e = launch_scaled_update(d, ms, gram, c->damping, g, mcores, acc, rule, dev_status, w + L.upd,
                                             L.ul, st);
            }
            if (e == hipSuccess) e = launch_bump(t_dev, st);
            if (e == hipSuccess && refresh)
                e = launch_dist(d, ModeSrc{nullptr, 0, n, 0}, false, n, c->law, live, p->cdf, dev_status, w + L.dist,
                                st);
        }
    }
    (void)rc;
    return hip_status(e);
}

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_addr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

// Device address of ``scratch`` on the current GPU, looked up once per GPU
// (with that GPU current) and kept.
hipError_t noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(g_scratch_once[dev], [dev]() {
        void* ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_addr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess) return g_scratch_err[dev];
    *out = g_scratch_addr[dev];
    return *out ? hipSuccess : hipErrorInvalidSymbol;
}

}  // namespace

extern "C" {

tr_status tr_run_noalloc(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps, double* loss_out,
                         int32_t* dev_status, tr_stream_t stream, const tr_run_opts* opts) {
    if (!p || !c || !t_dev) return TR_E_ARG;
    tr_status s = validate_desc(&p->desc);
    if (s != TR_OK) return s;
    if (c->m < 1 || c->m > kMaxM || c->m_H < 0 || c->m_H > kMaxM) return TR_E_SHAPE;
    if (run_layout(p, c).total > (size_t)TR_NOALLOC_SCRATCH_BYTES) return TR_E_WORKSPACE;
    void* ws = nullptr;
    if (noalloc_scratch(&ws) != hipSuccess) {
        (void)hipGetLastError();
        return TR_E_HIP;
    }
    return tr_run_ex(p, c, t_dev, steps, loss_out, dev_status, ws, (size_t)TR_NOALLOC_SCRATCH_BYTES, stream, opts);
}

size_t tr_batch_table_size(int32_t count) { return count > 0 ? align_up((size_t)count * sizeof(tr_batch_item)) : 0; }

tr_status tr_batch_upload(const tr_batch_item* items, int32_t count, void* table, size_t table_bytes,
                          tr_stream_t stream) {
    if (!items || count < 1 || count > 65535 || !table) return TR_E_ARG;
    if (table_bytes < tr_batch_table_size(count)) return TR_E_WORKSPACE;
    if (!aligned(table, 256)) return TR_E_ALIGN;
    for (int p = 0; p < count; ++p) {
        const tr_batch_item& it = items[p];
        const tr_desc& d = it.desc;
        tr_status s = validate_desc(&d);
        if (s != TR_OK) return s;
        if (d.core_dtype != TR_F32 || d.x_dtype != TR_F16) return TR_E_DTYPE;
        if (d.N > 5) return TR_E_SHAPE;
        if ((s = check_cores(&d, const_cast<const void* const*>(it.cores))) != TR_OK) return s;
        for (int k = 0; k < d.N; ++k) {
            if (d.I[k] > 128 || d.R[k] > 12) return TR_E_SHAPE;
            if (d.R[k] * d.R[(k + 1) % d.N] > 144) return TR_E_SHAPE;
            if (!it.Xrep[k]) return TR_E_ARG;
            if (it.rule.kind == 1 && !it.accum[k]) return TR_E_ARG;
        }
        if (!it.t_dev || it.m < 1 || it.m > kMaxM) return TR_E_ARG;
        if (it.rule.kind < 0 || it.rule.kind > 2) return TR_E_ARG;
        if (it.rule.kind == 2 && !(it.rule.tau > 0.0)) return TR_E_ARG;
    }
    return hip_status(hipMemcpyAsync(table, items, (size_t)count * sizeof(tr_batch_item), hipMemcpyHostToDevice,
                                     (hipStream_t)stream));
}

size_t tr_batch_split_workspace_size(int32_t count, int32_t splits) {
    if (count < 1 || count > 65535 || splits < 1 || splits > 16) return 0;
    return batch_split_ws_bytes(count, splits);
}

tr_status tr_batch_run_split(const void* table, int32_t count, int32_t steps, int32_t chunk, int32_t waves,
                             int32_t splits, void* ws, size_t ws_bytes, tr_stream_t stream) {
    if (!table || count < 1 || count > 65535 || steps < 0) return TR_E_ARG;
    if (!((chunk == 32 || chunk == 64) && (waves == 4 || waves == 8))) return TR_E_ARG;
    if (splits < 1 || splits > 16) return TR_E_ARG;
    if (!aligned(table, 256)) return TR_E_ALIGN;
    if (!ws || ws_bytes < batch_split_ws_bytes(count, splits)) return TR_E_WORKSPACE;
    if (!aligned(ws, 256)) return TR_E_ALIGN;
    if (steps == 0) return TR_OK;
    return hip_status(launch_batch_split(static_cast<const tr_batch_item*>(table), count, steps, chunk, waves, splits,
                                         ws, (hipStream_t)stream));
}

tr_status tr_batch_run(const void* table, int32_t count, int32_t steps, int32_t chunk, int32_t waves,
                       tr_stream_t stream) {
    if (!table || count < 1 || count > 65535 || steps < 0) return TR_E_ARG;
    if (!((chunk == 32 || chunk == 64) && (waves == 4 || waves == 8))) return TR_E_ARG;
    if (!aligned(table, 256)) return TR_E_ALIGN;
    if (steps == 0) return TR_OK;
    return hip_status(launch_batch_steps(static_cast<const tr_batch_item*>(table), count, steps, chunk, waves,
                                         (hipStream_t)stream));
}

}  // extern "C"
