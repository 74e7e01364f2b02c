// Host runtime of the solver: grid hierarchy and workspace plan, the V-cycle
// stage list (Algorithm 1 applied recursively), the refinement loop with
// residuum scaling (Algorithm 2), HIP-graph capture of one refinement step,
// and the C ABI declared in include/mgir.h.
#include "mgir.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mg_launch.h"

using namespace mg;

namespace {

thread_local std::string g_err;

mg_status_t fail(mg_status_t s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(x)                                                                               \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return fail(MG_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct LevelPlan {
    int n = 0, P = 0, prec = 0;
    size_t elems = 0;
    size_t off_b = 0, off_c[2] = {0, 0};
    Shape sh;       // smoothing, sweeps, prolongation
    Shape osh;      // refinement update (finest level only)
    RShape rsh;     // residual + restriction onto the next level
};

// One kernel launch recorded by the profiling mode.
struct ProfRec {
    const char *name;
    int level;
    double bytes;
    hipEvent_t a, b;
};

}  // namespace

struct mg_ctx {
    int dim = 3, n = 0, nl = 0;
    mg_options_t opt{};
    std::vector<LevelPlan> lv;
    size_t off_R = 0, off_U = 0, off_part = 0, off_scal = 0, ws_need = 0;
    int max_parts = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int cur[32] = {0};
    double *host_scal = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int outer_parts = 0;
    // profiling
    bool prof = false;
    std::vector<ProfRec> recs;
};

namespace {

template <class T> T *at_ws(mg_ctx *h, size_t off) { return reinterpret_cast<T *>(h->ws + off); }

void *cbuf(mg_ctx *h, int l, int which) { return h->ws + h->lv[l].off_c[which]; }
void *bbuf(mg_ctx *h, int l) { return h->ws + h->lv[l].off_b; }
double *Rbuf(mg_ctx *h) { return at_ws<double>(h, h->off_R); }
double *Ubuf(mg_ctx *h) { return at_ws<double>(h, h->off_U); }
double *part(mg_ctx *h) { return at_ws<double>(h, h->off_part); }
double *scal(mg_ctx *h) { return at_ws<double>(h, h->off_scal); }

long points(int D, int n) { return D == 3 ? (long)n * n * n : (long)n * n; }

bool valid_prec(int p) { return p >= 0 && p <= 3; }

Shape pick_shape(int D, int P, int prec) {
    Shape s;
    s.V = P >= 8 ? 8 : 4;
    s.bs = 256;
    s.xcd = 1;
    s.ty = 0;
    if (D == 3 && P >= 16) {
        // LDS-plane kernel: full rows, as many row groups as 1024 threads and
        // 64 KiB of LDS allow (at most 14 output rows)
        if (prec == P_F64) s.V = 4;
        const int TXR = P / s.V;
        int ty = std::min(14, P - 1);
        while (ty > 1 && (TXR * (ty + 2) > 1024 || march_lds_bytes(P, ty, prec_bytes(prec)) > 65536)) --ty;
        if (TXR * (ty + 2) <= 1024 && march_lds_bytes(P, ty, prec_bytes(prec)) <= 65536) {
            s.ty = ty;
            s.zc = std::max(1, std::min(8, P - 1));
            return s;
        }
    }
    const long per_chunk = (long)(P / s.V) * (D == 3 ? P : 1);
    const long target = 1L << 19;  // threads in flight: about 32 waves on each of 256 CUs
    const long nch = (target + per_chunk - 1) / per_chunk;
    int zc = (int)((P - 1 + nch - 1) / nch);
    s.zc = std::max(1, std::min(zc, 64));
    return s;
}

RShape pick_rshape(int D, int P, int pf) {
    RShape r;
    // eight FP64 values per thread exceed the register budget of a 1024-thread block
    r.V = (P >= 8 && pf != P_F64) ? 8 : 4;
    r.pipe = 0;
    if (D == 3 && P >= 16) {
        const int TXR = P / r.V, Pc = P / 2;
        const int pipe = TXR <= 64 ? 2 : 1;
        for (int tyc = std::min(7, Pc - 1); tyc >= 1; --tyc) {
            RShape c{r.V, tyc, 1, pipe};
            if ((2 * tyc + 3) * TXR <= 1024 && restrict_lds_bytes(D, P, pf, c) <= 65536) {
                const int ytiles = (Pc - 1 + tyc - 1) / tyc;
                const int nzc = std::max(1, (1024 + ytiles - 1) / ytiles);
                c.zcc = std::max(1, (Pc - 1 + nzc - 1) / nzc);
                return c;
            }
        }
    }
    const int TXR = P / r.V, Pc = P / 2;
    const size_t acc = pf == P_F64 ? 8 : 4;
    if (D == 3) {
        int tyc = 7;
        while (tyc > 1 && ((2 * tyc + 1) * TXR > 1024 || 2 * (size_t)(2 * tyc + 1) * P * acc > 65536)) --tyc;
        tyc = std::max(1, std::min(tyc, Pc - 1));
        r.tyc = tyc;
        const int ytiles = (Pc - 1 + tyc - 1) / tyc;
        const int nzc = std::max(1, (1024 + ytiles - 1) / ytiles);
        r.zcc = std::max(1, (Pc - 1 + nzc - 1) / nzc);
    } else {
        r.tyc = 1;
        r.zcc = std::max(1, (Pc - 1 + 63) / 64);
    }
    return r;
}

// ---- launch wrapper with optional per-launch events -------------------------
struct Launch {
    mg_ctx *h;
    hipStream_t st;
    const char *name;
    int level;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    Launch(mg_ctx *h_, hipStream_t st_, const char *nm, int lvl, double by) : h(h_), st(st_), name(nm), level(lvl), bytes(by) {
        if (h->prof) {
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            (void)hipEventRecord(a, st);
        }
    }
    hipError_t done(hipError_t e) {
        if (h->prof) {
            (void)hipEventRecord(b, st);
            h->recs.push_back(ProfRec{name, level, bytes, a, b});
        }
        return e;
    }
};

double sb(int prec) { return (double)prec_bytes(prec); }

#define RUN(h, st, name, lvl, bytes, call)                \
    do {                                                  \
        Launch L_((h), (st), (name), (lvl), (bytes));     \
        hipError_t e_ = L_.done(call);                    \
        if (e_ != hipSuccess) return e_;                  \
    } while (0)

// Pre-smoothing of level l from c = 0 into C[0] (plus extra sweeps), with the
// right-hand side taken from B_l, or for the finest level of a refinement step
// from the FP64 residual (scaled and cast on the fly, b-hat written to B_0).
hipError_t enq_presmooth(mg_ctx *h, hipStream_t st, int l, bool from_R) {
    LevelPlan &L = h->lv[l];
    const int D = h->dim;
    const double N = (double)points(D, L.n);
    const double s = sb(L.prec);
    const bool two = h->opt.nu1 >= 2;
    if (from_R) {
        RUN(h, st, two ? "smooth2_scaled" : "smooth1_scaled", l, N * (8 + 2 * s),
            launch_smooth_first(D, L.prec, L.P, nullptr, Rbuf(h), scal(h), bbuf(h, l), cbuf(h, l, 0), h->opt.omega,
                                two, L.sh, st));
    } else {
        RUN(h, st, two ? "smooth2" : "smooth1", l, N * 2 * s,
            launch_smooth_first(D, L.prec, L.P, bbuf(h, l), nullptr, nullptr, nullptr, cbuf(h, l, 0), h->opt.omega,
                                two, L.sh, st));
    }
    int cur = 0;
    for (int k = two ? 2 : 1; k < h->opt.nu1; ++k) {
        RUN(h, st, "sweep", l, N * 3 * s,
            launch_sweep(D, L.prec, L.P, bbuf(h, l), cbuf(h, l, cur), cbuf(h, l, cur ^ 1), h->opt.omega, L.sh, st));
        cur ^= 1;
    }
    h->cur[l] = cur;
    return hipSuccess;
}

hipError_t enq_restrict(mg_ctx *h, hipStream_t st, int l, const void *b) {
    LevelPlan &L = h->lv[l], &C = h->lv[l + 1];
    const double N = (double)points(h->dim, L.n);
    const double bytes = N * 2 * sb(L.prec) + (double)points(h->dim, C.n) * sb(C.prec);
    RUN(h, st, "resid_restrict", l, bytes,
        launch_restrict(h->dim, L.prec, C.prec, L.P, b, cbuf(h, l, h->cur[l]), bbuf(h, l + 1), L.rsh, st));
    return hipSuccess;
}

hipError_t enq_coarse(mg_ctx *h, hipStream_t st, int l) {
    LevelPlan &L = h->lv[l];
    RUN(h, st, "coarse_solve", l, 2 * sb(L.prec), launch_coarse(h->dim, L.prec, bbuf(h, l), cbuf(h, l, 0), st));
    h->cur[l] = 0;
    return hipSuccess;
}

hipError_t enq_prolong(mg_ctx *h, hipStream_t st, int l, const void *b) {
    LevelPlan &L = h->lv[l], &C = h->lv[l + 1];
    const double N = (double)points(h->dim, L.n);
    const double bytes = N * 3 * sb(L.prec) + (double)points(h->dim, C.n) * sb(C.prec);
    const int cur = h->cur[l];
    RUN(h, st, "prolong_sweep", l, bytes,
        launch_prolong(h->dim, L.prec, C.prec, L.P, cbuf(h, l, cur), cbuf(h, l + 1, h->cur[l + 1]), b,
                       cbuf(h, l, cur ^ 1), h->opt.omega, true, L.sh, st));
    h->cur[l] = cur ^ 1;
    return hipSuccess;
}

hipError_t enq_post(mg_ctx *h, hipStream_t st, int l, const void *b) {
    LevelPlan &L = h->lv[l];
    const double N = (double)points(h->dim, L.n);
    for (int k = 1; k < h->opt.nu2; ++k) {
        const int cur = h->cur[l];
        RUN(h, st, "sweep", l, N * 3 * sb(L.prec),
            launch_sweep(h->dim, L.prec, L.P, b, cbuf(h, l, cur), cbuf(h, l, cur ^ 1), h->opt.omega, L.sh, st));
        h->cur[l] = cur ^ 1;
    }
    return hipSuccess;
}

// Finest-level right-hand side modes of a V-cycle.
enum RhsMode { RHS_B = 0, RHS_SCALED_R = 1, RHS_ALIAS_R = 2 };

hipError_t enq_vcycle(mg_ctx *h, hipStream_t st, RhsMode mode) {
    const int nl = h->nl;
    std::vector<const void *> rhs(nl);
    for (int l = 0; l < nl; ++l) rhs[l] = bbuf(h, l);
    if (mode == RHS_ALIAS_R) rhs[0] = Rbuf(h);
    hipError_t e;
    for (int l = 0; l < nl - 1; ++l) {
        if (l == 0 && mode == RHS_ALIAS_R) {
            // FP64 baseline without scaling: the residual is the right-hand side
            LevelPlan &L = h->lv[0];
            const double N = (double)points(h->dim, L.n);
            const bool two = h->opt.nu1 >= 2;
            RUN(h, st, two ? "smooth2" : "smooth1", 0, N * 16,
                launch_smooth_first(h->dim, P_F64, L.P, Rbuf(h), nullptr, nullptr, nullptr, cbuf(h, 0, 0),
                                    h->opt.omega, two, L.sh, st));
            int cur = 0;
            for (int k = two ? 2 : 1; k < h->opt.nu1; ++k) {
                RUN(h, st, "sweep", 0, N * 24,
                    launch_sweep(h->dim, P_F64, L.P, Rbuf(h), cbuf(h, 0, cur), cbuf(h, 0, cur ^ 1), h->opt.omega,
                                 L.sh, st));
                cur ^= 1;
            }
            h->cur[0] = cur;
        } else {
            if ((e = enq_presmooth(h, st, l, l == 0 && mode == RHS_SCALED_R)) != hipSuccess) return e;
        }
        if ((e = enq_restrict(h, st, l, rhs[l])) != hipSuccess) return e;
    }
    if ((e = enq_coarse(h, st, nl - 1)) != hipSuccess) return e;
    for (int l = nl - 2; l >= 0; --l) {
        if ((e = enq_prolong(h, st, l, rhs[l])) != hipSuccess) return e;
        if ((e = enq_post(h, st, l, rhs[l])) != hipSuccess) return e;
    }
    return hipSuccess;
}

bool finest_alias(mg_ctx *h) { return h->lv[0].prec == P_F64 && !h->opt.residual_scaling; }

// One refinement step of Algorithm 2 (scale and cast, V-cycle, update) plus
// the norm readback.
hipError_t enq_step(mg_ctx *h, hipStream_t st) {
    hipError_t e = enq_vcycle(h, st, finest_alias(h) ? RHS_ALIAS_R : RHS_SCALED_R);
    if (e != hipSuccess) return e;
    LevelPlan &L = h->lv[0];
    const double hh = 1.0 / (double)(L.n + 1);
    const double N = (double)points(h->dim, L.n);
    RUN(h, st, "ir_update", 0, N * (32 + sb(L.prec)),
        launch_outer_update(h->dim, L.prec, L.P, cbuf(h, 0, h->cur[0]), Rbuf(h), Ubuf(h), scal(h), hh * hh, part(h),
                            L.osh, st));
    RUN(h, st, "norm_finalize", 0, 16.0 * h->outer_parts,
        launch_finalize(part(h), h->outer_parts, scal(h), h->opt.residual_scaling, st));
    return hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st);
}

void drop_graph(mg_ctx *h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}

mg_status_t ensure_graph(mg_ctx *h) {
    if (h->gexec) return MG_OK;
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enq_step(h, h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(MG_ERR_HIP, "capture of the refinement step failed: %s", hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(MG_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    h->graph = g;
    HIPCHK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    return MG_OK;
}

mg_status_t need_ws(mg_ctx *h) {
    if (!h) return fail(MG_ERR_ARG, "null handle");
    if (!h->ws) return fail(MG_ERR_WORKSPACE, "no workspace bound (call mg_bind_workspace)");
    return MG_OK;
}

int level_prec_code(int p) { return p; }


// ---- autotuner ------------------------------------------------------------
// Times candidate launch shapes of each level with HIP events on the caller's
// stream and keeps the fastest.  Every shape forms the same roundings, so the
// choice changes speed only.  Workspace contents are scratch at this point.
bool stencil_ok(const mg_ctx *h, const LevelPlan &L, const Shape &s) {
    if ((s.V != 4 && s.V != 8) || s.V > L.P || s.zc < 1 || s.zc > L.P - 1) return false;
    if (s.ty > 0) {
        if (h->dim != 3) return false;
        if ((L.P / s.V) * (s.ty + 2) > 1024 || march_lds_bytes(L.P, s.ty, prec_bytes(L.prec)) > 65536) return false;
        if (s.ty > L.P - 1) return false;
    }
    return true;
}

bool restrict_ok(const mg_ctx *h, const LevelPlan &L, const RShape &r) {
    const int Pc = L.P / 2;
    if ((r.V != 4 && r.V != 8) || r.V > L.P || r.zcc < 1 || r.zcc > std::max(1, Pc - 1)) return false;
    if (h->dim == 2 && (r.tyc != 1 || r.pipe)) return false;
    if (r.pipe < 0 || r.pipe > 2) return false;
    if (r.pipe == 2 && (L.P / r.V > 64 || r.V < 4)) return false;  // rows must not straddle waves
    if (r.tyc < 1 || r.tyc > std::max(1, Pc - 1)) return false;
    const int G = h->dim == 3 ? 2 * r.tyc + 1 + 2 * r.pipe : 1;
    if (G * (L.P / r.V) > 1024 || restrict_lds_bytes(h->dim, L.P, L.prec, r) > 65536) return false;
    if (L.prec == P_F64 && r.V == 8 && h->dim == 3) return false;  // spills registers
    return true;
}

template <class F> float time_ms(hipStream_t st, F &&fn, int reps) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    if (fn() != hipSuccess) return 1e30f;
    float best = 1e30f;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(a, st);
        if (fn() != hipSuccess) best = 1e30f;
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, a, b);
        best = std::min(best, t);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

std::vector<Shape> stencil_candidates(const mg_ctx *h, const LevelPlan &L, bool update) {
    std::vector<Shape> out;
    const int tys[] = {0, 2, 4, 6, 10, 14};
    const int zcs[] = {2, 4, 8, 16, 32, 64};
    for (int V : {4, 8})
        for (int ty : tys)
            for (int zc : zcs) {
                Shape s{V, zc, 256, 1, ty};
                if (ty == 0 && h->dim == 3 && zc < 8) continue;
                if (update && V == 8 && ty > 0) continue;  // FP64 rows spill at V = 8
                if (L.prec == P_F64 && V == 8 && ty > 0) continue;
                if (stencil_ok(h, L, s)) out.push_back(s);
            }
    return out;
}

mg_status_t autotune(mg_ctx *h, hipStream_t st) {
    const int D = h->dim;
    for (int l = 0; l + 1 < h->nl; ++l) {
        LevelPlan &L = h->lv[l];
        if (L.P < 8) continue;
        // smoothing family: first pre-smoothing + sweep + prolongation/sweep
        float best = 1e30f;
        Shape bs = L.sh;
        for (const Shape &s : stencil_candidates(h, L, false)) {
            L.sh = s;
            const float t = time_ms(st, [&]() -> hipError_t {
                hipError_t e = launch_smooth_first(D, L.prec, L.P, bbuf(h, l), nullptr, nullptr, nullptr,
                                                   cbuf(h, l, 0), h->opt.omega, true, s, st);
                if (e == hipSuccess)
                    e = launch_sweep(D, L.prec, L.P, bbuf(h, l), cbuf(h, l, 0), cbuf(h, l, 1), h->opt.omega, s, st);
                if (e == hipSuccess)
                    e = launch_prolong(D, L.prec, h->lv[l + 1].prec, L.P, cbuf(h, l, 1), cbuf(h, l + 1, 0),
                                       bbuf(h, l), cbuf(h, l, 0), h->opt.omega, true, s, st);
                return e;
            }, 3);
            if (t < best) best = t, bs = s;
        }
        L.sh = bs;
        // residual + restriction
        best = 1e30f;
        RShape br = L.rsh;
        for (int V : {4, 8})
            for (int tyc : {1, 2, 3, 4, 5, 7})
                for (int zcc : {2, 4, 8, 16, 32})
                    for (int pipe : {0, 1, 2}) {
                    RShape r{V, tyc, zcc, pipe};
                    if (!restrict_ok(h, L, r)) continue;
                    const float t = time_ms(st, [&]() {
                        return launch_restrict(D, L.prec, h->lv[l + 1].prec, L.P, bbuf(h, l), cbuf(h, l, 0),
                                               bbuf(h, l + 1), r, st);
                    }, 3);
                    if (t < best) best = t, br = r;
                }
        L.rsh = br;
        if (l == 0) {
            best = 1e30f;
            Shape bo = L.osh;
            const double hh = 1.0 / (double)(L.n + 1);
            for (const Shape &s : stencil_candidates(h, L, true)) {
                if (stencil_blocks(D, L.P, s) > h->max_parts) continue;
                const float t = time_ms(st, [&]() {
                    return launch_outer_update(D, L.prec, L.P, cbuf(h, 0, 0), Rbuf(h), Ubuf(h), scal(h), hh * hh,
                                               part(h), s, st);
                }, 3);
                if (t < best) best = t, bo = s;
            }
            L.osh = bo;
            h->outer_parts = stencil_blocks(D, L.P, bo);
        }
    }
    HIPCHK(hipMemsetAsync(h->ws, 0, h->ws_need, st));
    HIPCHK(hipStreamSynchronize(st));
    return MG_OK;
}
}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

void mg_default_options(mg_options_t *o) {
    if (!o) return;
    o->nu1 = 2;
    o->nu2 = 2;
    o->omega = 0.8;
    o->residual_scaling = 1;
    o->max_iter = 100;
    o->rtol = 1e-10;
    o->use_initial_guess = 0;
    o->use_graph = 1;
    o->autotune = 0;
}

const char *mg_status_string(mg_status_t s) {
    switch (s) {
    case MG_OK: return "ok";
    case MG_ERR_ARG: return "invalid argument";
    case MG_ERR_SHAPE: return "invalid grid shape";
    case MG_ERR_PREC: return "invalid precision";
    case MG_ERR_WORKSPACE: return "workspace missing or too small";
    case MG_ERR_HIP: return "HIP runtime error";
    case MG_ERR_NOT_CONVERGED: return "not converged";
    case MG_ERR_NONFINITE: return "non-finite residual";
    case MG_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char *mg_last_error(void) { return g_err.c_str(); }

mg_status_t mg_setup(mg_handle *out, int dim, int n, int nlevels, const mg_prec_t *level_prec,
                     const mg_options_t *opt) {
    if (!out) return fail(MG_ERR_ARG, "out is null");
    if (dim != 2 && dim != 3) return fail(MG_ERR_SHAPE, "dim must be 2 or 3, got %d", dim);
    if (n < 3 || ((n + 1) & n) != 0 || n > 4095)
        return fail(MG_ERR_SHAPE, "n must be 2^m - 1 with 2 <= m <= 12, got %d", n);
    if (dim == 3 && n > 1023)
        return fail(MG_ERR_SHAPE, "3-D grids are limited to n <= 1023 (one block must hold three fine rows)");
    int m = 0;
    while ((1 << m) < n + 1) ++m;
    if (nlevels != 0 && nlevels != m)
        return fail(MG_ERR_ARG, "nlevels must be 0 or %d (the full hierarchy down to one point), got %d", m, nlevels);
    mg_options_t o;
    mg_default_options(&o);
    if (opt) o = *opt;
    if (o.nu1 < 1 || o.nu1 > 16 || o.nu2 < 1 || o.nu2 > 16)
        return fail(MG_ERR_ARG, "nu1 and nu2 must be in 1..16 (got %d, %d)", o.nu1, o.nu2);
    if (!(o.omega > 0.0 && o.omega < 2.0)) return fail(MG_ERR_ARG, "omega must be in (0, 2)");
    if (o.max_iter < 0) return fail(MG_ERR_ARG, "max_iter must be >= 0");
    if (!(o.rtol >= 0.0)) return fail(MG_ERR_ARG, "rtol must be >= 0");
    std::vector<int> prec(m, P_F64);
    if (level_prec)
        for (int i = 0; i < m; ++i) {
            if (!valid_prec((int)level_prec[i])) return fail(MG_ERR_PREC, "level_prec[%d] = %d is not a format", i, (int)level_prec[i]);
            prec[i] = (int)level_prec[i];
        }
    mg_ctx *h = new mg_ctx();
    h->dim = dim;
    h->n = n;
    h->nl = m;
    h->opt = o;
    h->lv.resize(m);
    size_t off = 0;
    int nn = n;
    int maxp = 0;
    for (int l = 0; l < m; ++l) {
        LevelPlan &L = h->lv[l];
        L.n = nn;
        L.P = nn + 1;
        L.prec = prec[l];
        L.elems = level_elems(dim, L.P);
        const size_t bytes = align_up(L.elems * prec_bytes(L.prec), 256);
        L.off_b = off;
        off += bytes;
        L.off_c[0] = off;
        off += bytes;
        L.off_c[1] = off;
        off += bytes;
        if (nn > 1) {
            L.sh = pick_shape(dim, L.P, L.prec);
            L.osh = pick_shape(dim, L.P, P_F64);  // FP64 rows dominate the update's registers
            L.rsh = pick_rshape(dim, L.P, L.prec);
        }
        nn = (nn - 1) / 2;
    }
    const size_t fin = align_up(h->lv[0].elems * sizeof(double), 256);
    h->off_R = off;
    off += fin;
    h->off_U = off;
    off += fin;
    if (m > 1) {
        h->outer_parts = stencil_blocks(dim, h->lv[0].P, h->lv[0].osh);
        // room for the partials of any legal shape: V = 4, zc = 1, 64-thread blocks
        const int P0 = h->lv[0].P;
        const long worst = ((long)(P0 / 4) * (dim == 3 ? P0 : 1) * (P0 - 1) + 63) / 64;
        maxp = (int)std::max<long>(h->outer_parts, worst);
    }
    maxp = std::max(maxp, flat_blocks(points(dim, n)));
    h->max_parts = maxp;
    h->off_part = off;
    off += align_up((size_t)maxp * 2 * sizeof(double), 256);
    h->off_scal = off;
    off += 256;
    h->ws_need = off;
    *out = h;
    return MG_OK;
}

mg_status_t mg_workspace_size(mg_handle h, size_t *bytes) {
    if (!h || !bytes) return fail(MG_ERR_ARG, "null argument");
    *bytes = h->ws_need;
    return MG_OK;
}

mg_status_t mg_bind_workspace(mg_handle h, void *dev_ptr, size_t bytes, void *stream) {
    if (!h || !dev_ptr) return fail(MG_ERR_ARG, "null argument");
    if (bytes < h->ws_need) return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes < %zu needed", bytes, h->ws_need);
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(MG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!h->host_scal) HIPCHK(hipHostMalloc((void **)&h->host_scal, 4 * sizeof(double), hipHostMallocDefault));
    drop_graph(h);
    h->ws = static_cast<char *>(dev_ptr);
    h->ws_bytes = bytes;
    HIPCHK(hipMemsetAsync(h->ws, 0, h->ws_need, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int l = 0; l < h->nl; ++l) h->cur[l] = 0;
    if (h->opt.autotune) {
        mg_status_t s = autotune(h, st);
        if (s != MG_OK) return s;
    }
    return MG_OK;
}

mg_status_t mg_destroy(mg_handle h) {
    if (!h) return MG_OK;
    drop_graph(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->host_scal) (void)hipHostFree(h->host_scal);
    delete h;
    return MG_OK;
}

mg_status_t mg_levels(mg_handle h, int *nlevels) {
    if (!h || !nlevels) return fail(MG_ERR_ARG, "null argument");
    *nlevels = h->nl;
    return MG_OK;
}

mg_status_t mg_level_n(mg_handle h, int level, int *n) {
    if (!h || !n) return fail(MG_ERR_ARG, "null argument");
    if (level < 0 || level >= h->nl) return fail(MG_ERR_ARG, "level %d out of range", level);
    *n = h->lv[level].n;
    return MG_OK;
}

static mg_status_t buffer_of(mg_ctx *h, int level, mg_buffer_t buf, void **p, int *prec) {
    if (level < 0 || level >= h->nl) return fail(MG_ERR_ARG, "level %d out of range", level);
    switch (buf) {
    case MG_BUF_RHS: *p = bbuf(h, level); *prec = h->lv[level].prec; return MG_OK;
    case MG_BUF_COR: *p = cbuf(h, level, h->cur[level]); *prec = h->lv[level].prec; return MG_OK;
    case MG_BUF_RES:
        if (level != 0) return fail(MG_ERR_ARG, "MG_BUF_RES exists on level 0 only");
        *p = Rbuf(h); *prec = P_F64; return MG_OK;
    case MG_BUF_SOL:
        if (level != 0) return fail(MG_ERR_ARG, "MG_BUF_SOL exists on level 0 only");
        *p = Ubuf(h); *prec = P_F64; return MG_OK;
    }
    return fail(MG_ERR_ARG, "unknown buffer %d", (int)buf);
}

mg_status_t mg_level_write(mg_handle h, int level, mg_buffer_t buf, const void *src, mg_prec_t src_prec,
                           void *stream) {
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!src) return fail(MG_ERR_ARG, "src is null");
    if (!valid_prec(src_prec)) return fail(MG_ERR_PREC, "src_prec %d", (int)src_prec);
    void *p;
    int prec;
    if ((s = buffer_of(h, level, buf, &p, &prec)) != MG_OK) return s;
    HIPCHK(launch_pack(h->dim, src_prec, prec, h->lv[level].n, h->lv[level].P, src, p,
                       static_cast<hipStream_t>(stream)));
    return MG_OK;
}

mg_status_t mg_level_read(mg_handle h, int level, mg_buffer_t buf, void *dst, mg_prec_t dst_prec, void *stream) {
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!dst) return fail(MG_ERR_ARG, "dst is null");
    if (!valid_prec(dst_prec)) return fail(MG_ERR_PREC, "dst_prec %d", (int)dst_prec);
    void *p;
    int prec;
    if ((s = buffer_of(h, level, buf, &p, &prec)) != MG_OK) return s;
    HIPCHK(launch_unpack(h->dim, prec, dst_prec, h->lv[level].n, h->lv[level].P, p, dst,
                         static_cast<hipStream_t>(stream)));
    return MG_OK;
}

mg_status_t mg_stage(mg_handle h, mg_stage_t stage, int level, void *stream) {
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (level < 0 || level >= h->nl) return fail(MG_ERR_ARG, "level %d out of range", level);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool base = level == h->nl - 1;
    hipError_t e = hipSuccess;
    switch (stage) {
    case MG_STAGE_SMOOTH_FIRST:
        if (base) return fail(MG_ERR_ARG, "the base level is solved, not smoothed");
        e = enq_presmooth(h, st, level, false);
        break;
    case MG_STAGE_SWEEP: {
        if (base) return fail(MG_ERR_ARG, "the base level is solved, not smoothed");
        LevelPlan &L = h->lv[level];
        const int cur = h->cur[level];
        e = launch_sweep(h->dim, L.prec, L.P, bbuf(h, level), cbuf(h, level, cur), cbuf(h, level, cur ^ 1),
                         h->opt.omega, L.sh, st);
        if (e == hipSuccess) h->cur[level] = cur ^ 1;
        break;
    }
    case MG_STAGE_RESTRICT:
        if (base) return fail(MG_ERR_ARG, "the base level has no coarser level");
        e = enq_restrict(h, st, level, bbuf(h, level));
        break;
    case MG_STAGE_PROLONG_SWEEP:
        if (base) return fail(MG_ERR_ARG, "the base level has no coarser level");
        e = enq_prolong(h, st, level, bbuf(h, level));
        break;
    case MG_STAGE_COARSE:
        if (!base) return fail(MG_ERR_ARG, "MG_STAGE_COARSE applies to the base level (%d)", h->nl - 1);
        e = enq_coarse(h, st, level);
        break;
    default:
        return fail(MG_ERR_ARG, "unknown stage %d", (int)stage);
    }
    if (e != hipSuccess) return fail(MG_ERR_HIP, "stage launch failed: %s", hipGetErrorString(e));
    return MG_OK;
}

mg_status_t mg_vcycle(mg_handle h, const void *b, void *c, void *stream) {
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!b || !c) return fail(MG_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    LevelPlan &L = h->lv[0];
    HIPCHK(launch_pack(h->dim, L.prec, L.prec, L.n, L.P, b, bbuf(h, 0), st));
    HIPCHK(enq_vcycle(h, st, RHS_B));
    HIPCHK(launch_unpack(h->dim, L.prec, L.prec, L.n, L.P, cbuf(h, 0, h->cur[0]), c, st));
    return MG_OK;
}

mg_status_t ir_solve(mg_handle h, const double *b, double *u, mg_stats_t *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!b || !u) return fail(MG_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    LevelPlan &L = h->lv[0];
    const double hh = 1.0 / (double)(L.n + 1);
    const double inv_h2 = 1.0 / (hh * hh);
    const int D = h->dim;
    const int scaling = h->opt.residual_scaling;
    auto finish_stats = [&](int iters, double rel) {
        if (stats) {
            stats->iterations = iters;
            stats->rel_residual = rel;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
    };
    auto hist = [&](int k, double v) {
        if (stats && stats->history && k < stats->history_cap) stats->history[k] = v;
    };

    // ||b||_2 first (and the initial residual when u starts at zero)
    if (h->opt.use_initial_guess) {
        HIPCHK(launch_resid_flat(D, L.n, L.P, b, nullptr, nullptr, nullptr, inv_h2, part(h), st));
    } else {
        HIPCHK(launch_resid_flat(D, L.n, L.P, b, nullptr, Rbuf(h), nullptr, inv_h2, part(h), st));
        HIPCHK(launch_fill_zero(Ubuf(h), align_up(L.elems * sizeof(double), 16), st));
    }
    const int fparts = flat_blocks(points(D, L.n));
    HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
    HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double nb = h->host_scal[2];
    if (!std::isfinite(nb)) {
        finish_stats(0, NAN);
        return fail(MG_ERR_NONFINITE, "||b|| is not finite");
    }
    if (nb == 0.0) {
        HIPCHK(hipMemsetAsync(u, 0, sizeof(double) * points(D, L.n), st));
        HIPCHK(hipStreamSynchronize(st));
        hist(0, 0.0);
        finish_stats(0, 0.0);
        return MG_OK;
    }
    if (h->opt.use_initial_guess) {
        HIPCHK(launch_pack(D, P_F64, P_F64, L.n, L.P, u, Ubuf(h), st));
        HIPCHK(launch_resid_flat(D, L.n, L.P, b, Ubuf(h), Rbuf(h), nullptr, inv_h2, part(h), st));
        HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
        HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    const bool graph = h->opt.use_graph && !h->prof;
    if (graph) {
        s = ensure_graph(h);
        if (s != MG_OK) return s;
    }
    int k = 0;
    bool recursive = false;  // whether R holds a recursively updated residual
    mg_status_t result = MG_OK;
    double rel = h->host_scal[2] / nb;
    for (;;) {
        const double rn = h->host_scal[2];
        rel = rn / nb;
        hist(k, rel);
        if (!std::isfinite(rn)) {
            result = fail(MG_ERR_NONFINITE, "residual norm became non-finite at iteration %d", k);
            break;
        }
        if (rn <= h->opt.rtol * nb) {
            if (!recursive) break;
            // confirm with the residual recomputed from u
            HIPCHK(launch_resid_flat(D, L.n, L.P, b, Ubuf(h), Rbuf(h), u, inv_h2, part(h), st));
            HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
            HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            recursive = false;
            rel = h->host_scal[2] / nb;
            hist(k, rel);
            if (h->host_scal[2] <= h->opt.rtol * nb) {
                finish_stats(k, rel);
                return MG_OK;  // u already written by the confirmation pass
            }
            continue;
        }
        if (k >= h->opt.max_iter) {
            result = fail(MG_ERR_NOT_CONVERGED, "not converged in %d iterations (rel. residual %.3e)", k, rel);
            break;
        }
        if (graph) {
            HIPCHK(hipGraphLaunch(h->gexec, st));
        } else {
            hipError_t e = enq_step(h, st);
            if (e != hipSuccess) return fail(MG_ERR_HIP, "refinement step launch failed: %s", hipGetErrorString(e));
        }
        HIPCHK(hipStreamSynchronize(st));
        recursive = true;
        ++k;
    }
    // final: recompute the true residual and copy u out
    HIPCHK(launch_resid_flat(D, L.n, L.P, b, Ubuf(h), Rbuf(h), u, inv_h2, part(h), st));
    HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
    HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rel = h->host_scal[2] / nb;
    finish_stats(k, rel);
    return result;
}

mg_status_t mg_set_shape(mg_handle h, int level, int kind, const int *p, int np) {
    if (!h || !p) return fail(MG_ERR_ARG, "null argument");
    if (level < 0 || level >= h->nl - 1) return fail(MG_ERR_ARG, "level %d has no launch shape", level);
    LevelPlan &L = h->lv[level];
    const int D = h->dim;
    if (kind == MG_SHAPE_STENCIL || kind == MG_SHAPE_UPDATE) {
        if (kind == MG_SHAPE_UPDATE && level != 0) return fail(MG_ERR_ARG, "the update shape exists on level 0 only");
        if (np != 5) return fail(MG_ERR_ARG, "stencil shape takes 5 values {V, zc, bs, xcd, ty}");
        Shape s{p[0], p[1], p[2], p[3], p[4]};
        if ((s.V != 4 && s.V != 8) || s.V > L.P) return fail(MG_ERR_ARG, "V must be 4 or 8 and <= P = %d", L.P);
        if (s.zc < 1 || s.zc > L.P) return fail(MG_ERR_ARG, "zc out of range");
        if (s.bs < 64 || s.bs > 256 || s.bs % 64) return fail(MG_ERR_ARG, "bs must be 64, 128, 192 or 256");
        if (s.xcd != 0 && s.xcd != 1) return fail(MG_ERR_ARG, "xcd must be 0 or 1");
        if (s.ty < 0 || (D == 2 && s.ty != 0)) return fail(MG_ERR_ARG, "ty must be 0 (2-D) or >= 0 (3-D)");
        if (s.ty > 0 && ((L.P / s.V) * (s.ty + 2) > 1024 || march_lds_bytes(L.P, s.ty, prec_bytes(L.prec)) > 65536))
            return fail(MG_ERR_ARG, "ty = %d exceeds 1024 threads or 64 KiB of LDS", s.ty);
        if (kind == MG_SHAPE_UPDATE) {
            if (stencil_blocks(D, L.P, s) > h->max_parts) return fail(MG_ERR_ARG, "too many blocks");
            L.osh = s;
            h->outer_parts = stencil_blocks(D, L.P, s);
        } else {
            L.sh = s;
        }
    } else if (kind == MG_SHAPE_RESTRICT) {
        if (np != 4) return fail(MG_ERR_ARG, "restriction shape takes 4 values {V, tyc, zcc, pipe}");
        RShape r{p[0], p[1], p[2], p[3]};
        if (!restrict_ok(h, L, r))
            return fail(MG_ERR_ARG, "restriction shape {%d, %d, %d, %d} is not valid on level %d", r.V, r.tyc,
                        r.zcc, r.pipe, level);
        L.rsh = r;
    } else {
        return fail(MG_ERR_ARG, "unknown shape kind %d", kind);
    }
    drop_graph(h);
    return MG_OK;
}

mg_status_t mg_get_shape(mg_handle h, int level, int kind, int *p, int np) {
    if (!h || !p) return fail(MG_ERR_ARG, "null argument");
    if (level < 0 || level >= h->nl - 1) return fail(MG_ERR_ARG, "level %d has no launch shape", level);
    const LevelPlan &L = h->lv[level];
    if ((kind == MG_SHAPE_STENCIL || (kind == MG_SHAPE_UPDATE && level == 0)) && np >= 5) {
        const Shape &S = kind == MG_SHAPE_STENCIL ? L.sh : L.osh;
        p[0] = S.V, p[1] = S.zc, p[2] = S.bs, p[3] = S.xcd, p[4] = S.ty;
    } else if (kind == MG_SHAPE_RESTRICT && np >= 4) {
        p[0] = L.rsh.V, p[1] = L.rsh.tyc, p[2] = L.rsh.zcc, p[3] = L.rsh.pipe;
    } else {
        return fail(MG_ERR_ARG, "bad kind or too few values");
    }
    return MG_OK;
}

mg_status_t mg_bandwidth_probe(void *dst, const void *src, size_t bytes, int kind, int blocks, void *stream) {
    if (!dst || !src || kind < 0 || kind > 2 || blocks < 1) return fail(MG_ERR_ARG, "bad argument");
    if (bytes % 16) return fail(MG_ERR_ARG, "bytes must be a multiple of 16");
    HIPCHK(launch_probe(dst, src, bytes, kind, blocks, static_cast<unsigned *>(dst), static_cast<hipStream_t>(stream)));
    return MG_OK;
}

mg_status_t mg_profile_step(mg_handle h, void *stream, int cap, int *count, const char **names, double *ms,
                            double *bytes, int *levels_out) {
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!count || cap < 0) return fail(MG_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    h->prof = true;
    h->recs.clear();
    hipError_t e = enq_step(h, st);
    h->prof = false;
    hipError_t e2 = hipStreamSynchronize(st);
    int i = 0;
    for (auto &r : h->recs) {
        float t = 0.f;
        (void)hipEventElapsedTime(&t, r.a, r.b);
        if (i < cap) {
            if (names) names[i] = r.name;
            if (ms) ms[i] = t;
            if (bytes) bytes[i] = r.bytes;
            if (levels_out) levels_out[i] = r.level;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        ++i;
    }
    *count = i;
    h->recs.clear();
    if (e != hipSuccess) return fail(MG_ERR_HIP, "profiled step failed: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(MG_ERR_HIP, "profiled step failed: %s", hipGetErrorString(e2));
    return MG_OK;
}

}  // extern "C"
