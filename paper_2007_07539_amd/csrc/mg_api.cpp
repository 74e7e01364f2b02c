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
#include <cstdlib>
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

enum { SH_SMOOTH = 0, SH_SWEEP = 1, SH_PROLONG = 2 };

struct LevelPlan {
    int n = 0, P = 0, prec = 0;
    size_t elems = 0;
    size_t off_b = 0, off_c[2] = {0, 0};
    size_t off_cg = 0;     // CG vectors of a multi-point base level
    // fused first smoothing + restriction from the stored b (levels >= 1)
    bool fsr_on = true, fsr = false;
    RShape fsrsh{8, 2, 16, 3};
    bool rescale = false;  // restrictions into this level rescale (half-precision level, rescale_half)
    size_t off_t = 0;      // its restricted residual / scaled correction in the finer accumulator format
    Shape shs[3];   // kernel families: SH_SMOOTH (first pre-smoothing), SH_SWEEP, SH_PROLONG
    Shape osh;      // refinement update (finest level only)
    RShape rsh;     // residual + restriction onto the next level
    Q1Shape q1s[3];  // Q1: the LDS-staged sweep, residual and update (finest level only); {0, 0}: built-in
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
    // finalize-kernel code of the residual scaling: 0 = off (alpha = 1),
    // 1 + j = on with alpha = 2^j ||r||_inf (see alpha_shift)
    int ascale = 0;
    std::vector<LevelPlan> lv;
    size_t off_R = 0, off_U = 0, off_part = 0, off_scal = 0, ws_need = 0;
    size_t vc_bytes = 0;  // the leading part of the workspace a lone V-cycle uses
    size_t off_rs = 0, off_rpart = 0;  // per-level {s, 1/s} and the partial maxima of the rescaling
    int max_parts = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int cur[32] = {0};
    double *host_scal = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph2 = nullptr;      // single grid: the update part of a step
    hipGraphExec_t gexec2 = nullptr;
    // single grid whose update swaps the residual arrays (see swaps_r): the
    // two graphs of a step that starts from the second array
    hipGraph_t graph_p1 = nullptr, graph2_p1 = nullptr;
    hipGraphExec_t gexec_p1 = nullptr, gexec2_p1 = nullptr;
    size_t off_R2 = 0;  // the second residual array (0: none)
    int rpar = 0;       // 1: the current residual is in the second array
    // postponed solution updates (opt.defer_update)
    int defer = 0;      // ring depth in use; 0: u is updated every step
    size_t off_cdef = 0, cdef_stride = 0, off_adef = 0, off_dctr = 0;
    int pending = 0;    // corrections in the ring not yet added to u
    bool u_zero = false;  // u is zero and not yet stored (a solve from zero with postponed updates)
    hipEvent_t ev_norm = nullptr;     // single grid: the norm readback of a step is done
    int outer_parts = 0;
    bool tail_on = true;
    bool q1 = false;       // Q1 finite elements (mg_q1.hip kernels) instead of finite differences
    size_t off_q1r = 0;    // Q1: fine residual ahead of its restriction (any level's, accumulator format)
    bool fuse_on = true;   // allow the fused last sweep + update on the finest level
    bool fused = false;    // ... and it is in use
    Shape fsh{4, 16, 256, 1, 4};
    bool su_r = true;      // ... forming b from r (else reading b back); needs the second residual array
    bool fuse_sr_on = true;  // allow the fused first smoothing + restriction on the finest level
    bool fused_sr = false;   // ... and it is in use
    RShape srsh{8, 2, 16, 3};
    // profiling
    bool prof = false;
    std::vector<ProfRec> recs;
    // batched instances
    bool batched = false;
    struct Inst {
        int n = 0, nl = 0;
        std::vector<LevelPlan> lv;
        size_t off_R = 0, off_U = 0;
        int part_off = 0, parts = 0;
        Shape osh;
        int ascale = 0;
    };
    std::vector<Inst> inst;
    int Lmax = 0;
    std::vector<int> bprec;  // batched level map (finest first, last = base)
    struct BLaunch {
        int what;  // 0 stencil, 1 restriction, 2 base solve, 3 finalize
        int kind, V, pf, pc;
        size_t off_desc, off_items;
        int ndesc, nitems, grid, threads;
        size_t lds;
        const char *name;
        int level;
        double bytes;
    };
    std::vector<BLaunch> bl;
    size_t off_bmeta = 0, bmeta_bytes = 0, off_active = 0, off_scal_all = 0, off_fin = 0;
    size_t bmeta_cap = 0;  // workspace bytes reserved for the descriptor image
    int *host_active = nullptr;
    double *host_scal_all = nullptr;
    std::vector<unsigned char> bmeta_img_tmp;
    // many right-hand sides (interleaved); nrhs == 0 for other handles
    int nrhs = 0;
    size_t off_act = 0, off_mask = 0, off_zmask = 0, off_mres = 0;
    int m_upd_blocks = 0;
    int *host_mask = nullptr;
    double *host_scal_m = nullptr;
};

namespace {

template <class T> T *at_ws(mg_ctx *h, size_t off) { return reinterpret_cast<T *>(h->ws + off); }

void *cbuf(mg_ctx *h, int l, int which) { return h->ws + h->lv[l].off_c[which]; }
void *bbuf(mg_ctx *h, int l) { return h->ws + h->lv[l].off_b; }
// The current residual, and (FP64 map without scaling, fused update) the
// array the next update writes.
double *Rbuf(mg_ctx *h) { return at_ws<double>(h, h->rpar ? h->off_R2 : h->off_R); }
double *Rnext(mg_ctx *h) { return at_ws<double>(h, h->rpar ? h->off_R : h->off_R2); }
double *Ubuf(mg_ctx *h) { return at_ws<double>(h, h->off_U); }
double *part(mg_ctx *h) { return at_ws<double>(h, h->off_part); }
double *scal(mg_ctx *h) { return at_ws<double>(h, h->off_scal); }
double *rscal(mg_ctx *h, int l) { return at_ws<double>(h, h->off_rs) + 2 * l; }
// accumulator format of level l's arithmetic (the format a rescaled
// restriction out of level l keeps before the cast)
int acc_prec(int prec) { return prec == P_F64 ? P_F64 : P_F32; }
bool half_prec(int prec) { return prec == P_F16 || prec == P_BF16; }

long points(int D, int n) { return D == 3 ? (long)n * n * n : (long)n * n; }
// Largest base level the one-workgroup CG solves (64^3 points).
constexpr long kMaxBasePoints = 262144;
// Deepest ring of postponed solution updates.
constexpr int kMaxDefer = 64;

bool valid_prec(int p) { return p >= 0 && p <= 3; }

// Range of the FP16 levels.  Residual scaling divides r by alpha = ||r||_inf
// so that the correction equation's right-hand side has max-norm one
// (Algorithm 2).  Its solution in grid-scaled units on a level of n points per
// dimension is then bounded by max(L^-1 1) (discrete maximum principle), which
// is close to w_D (n + 1)^2 with w_D the centre value of the torsion function
// of the unit square, 0.07367, or cube, 0.05621: the finite-difference values
// approach it from below, the Q1 values (lumped unit load) from above, and
// K_D = 0.074 (2-D), 0.058 (3-D) bounds both on every grid of 15 or more points
// per dimension.  From about 2^14 on (2-D n >= 511, 3-D n = 1023) a V-cycle's
// values would come within a factor four of FP16's largest value 65504, or
// beyond it.  The scale is then alpha = 2^j ||r||_inf with the least j that
// brings K_D (n + 1)^2 of every FP16 level under 2^14; a power of two, so
// nothing else in the method changes.
constexpr double kHalfCorrectionBound = 16384.0;
double correction_bound(int D, int n) { return (D == 2 ? 0.074 : 0.058) * (double)(n + 1) * (double)(n + 1); }
int shift_for_bound(double bound) {
    int j = 0;
    while (bound > kHalfCorrectionBound * std::ldexp(1.0, j)) ++j;
    return j;
}
// Finalize code (0: alpha = 1; 1 + j: alpha = 2^j ||r||_inf) of a hierarchy
// with sizes ns[l] and formats prec[l], finest first.  A level entered by a
// rescaled restriction (rescaled[l]) has its own right-hand side of max-norm
// one, which alpha does not change: its bound must hold as it is (false).
bool alpha_code(int D, const std::vector<int> &ns, const std::vector<int> &prec, const std::vector<bool> &rescaled,
                int scaling, int *code) {
    int j = 0;
    for (size_t l = 0; l < ns.size(); ++l) {
        if (prec[l] != P_F16) continue;
        const double bnd = correction_bound(D, ns[l]);
        if (rescaled[l]) {
            if (bnd > kHalfCorrectionBound) return false;
        } else {
            j = std::max(j, shift_for_bound(bnd));
        }
    }
    *code = scaling ? 1 + j : 0;
    return true;
}

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

// Launches that differ between the discretisations.  The Q1 forms have no
// fused variants (mg_q1.hip); their shapes are those of the LDS-staged kernels.
hipError_t level_sweep(mg_ctx *h, int l, int prec, const void *b, const void *c, void *c_out, hipStream_t st) {
    const LevelPlan &L = h->lv[l];
    if (h->q1) return launch_q1_sweep(h->dim, prec, L.n, L.P, b, c, c_out, h->opt.omega, st, L.q1s[0]);
    return launch_sweep(h->dim, prec, L.P, b, c, c_out, h->opt.omega, L.shs[SH_SWEEP], st);
}

hipError_t level_first(mg_ctx *h, int l, int prec, const void *b, const double *r, const double *sc, void *b_out,
                       void *c_out, bool two, hipStream_t st) {
    const LevelPlan &L = h->lv[l];
    if (h->q1) return launch_q1_first(h->dim, prec, L.n, L.P, b, r, sc, b_out, c_out, h->opt.omega, st);
    return launch_smooth_first(h->dim, prec, L.P, b, r, sc, b_out, c_out, h->opt.omega, two, L.shs[SH_SMOOTH], st);
}

hipError_t level_restrict(mg_ctx *h, int l, int pf, int pc, const void *b, const void *c, void *bc, hipStream_t st) {
    const LevelPlan &L = h->lv[l];
    if (h->q1) return launch_q1_restrict(h->dim, pf, pc, L.n, L.P, b, c, h->ws + h->off_q1r, bc, st, L.q1s[1]);
    return launch_restrict(h->dim, pf, pc, L.P, b, c, bc, L.rsh, st);
}

hipError_t level_prolong(mg_ctx *h, int l, int pf, int pc, const void *c, const void *ec, const void *b, void *c_out,
                         hipStream_t st) {
    const LevelPlan &L = h->lv[l];
    if (h->q1) return launch_q1_prolong(h->dim, pf, pc, L.n, L.P, c, ec, b, c_out, h->opt.omega, st, L.q1s[0]);
    return launch_prolong(h->dim, pf, pc, L.P, c, ec, b, c_out, h->opt.omega, true, L.shs[SH_PROLONG], st);
}

// r = b - A U on the finest level from the dense b (see launch_resid_flat).
hipError_t finest_resid(mg_ctx *h, const double *b, const double *U, double *R, double *uout, hipStream_t st) {
    const LevelPlan &L = h->lv[0];
    const double hh = 1.0 / (double)(L.n + 1);
    if (h->q1)
        return launch_q1_resid_flat(h->dim, L.n, L.P, b, U, R, uout, h->dim == 3 ? hh : 1.0, part(h), st);
    return launch_resid_flat(h->dim, L.n, L.P, b, U, R, uout, 1.0 / (hh * hh), part(h), st);
}

// Pre-smoothing of level l from c = 0 into C[0] (plus extra sweeps), with the
// right-hand side taken from B_l, or for the finest level of a refinement step
// from the FP64 residual (scaled and cast on the fly, b-hat written to B_0).
hipError_t enq_presmooth(mg_ctx *h, hipStream_t st, int l, bool from_R) {
    LevelPlan &L = h->lv[l];
    const int D = h->dim;
    const double N = (double)points(D, L.n);
    const double s = sb(L.prec);
    const bool two = h->opt.nu1 >= 2 && !h->q1;
    (void)D;
    if (from_R) {
        RUN(h, st, two ? "smooth2_scaled" : "smooth1_scaled", l, N * (8 + 2 * s),
            level_first(h, l, L.prec, nullptr, Rbuf(h), scal(h), bbuf(h, l), cbuf(h, l, 0), two, st));
    } else {
        RUN(h, st, two ? "smooth2" : "smooth1", l, N * 2 * s,
            level_first(h, l, L.prec, bbuf(h, l), nullptr, nullptr, nullptr, cbuf(h, l, 0), two, st));
    }
    int cur = 0;
    for (int k = two ? 2 : 1; k < h->opt.nu1; ++k) {
        RUN(h, st, "sweep", l, N * 3 * s, level_sweep(h, l, L.prec, bbuf(h, l), cbuf(h, l, cur), cbuf(h, l, cur ^ 1), st));
        cur ^= 1;
    }
    h->cur[l] = cur;
    return hipSuccess;
}

hipError_t enq_restrict(mg_ctx *h, hipStream_t st, int l, const void *b) {
    LevelPlan &L = h->lv[l], &C = h->lv[l + 1];
    const double N = (double)points(h->dim, L.n);
    const double bytes = N * 2 * sb(L.prec) + (double)points(h->dim, C.n) * sb(C.prec);
    if (C.rescale) {
        // restrict in the fine accumulator format, then s = max |t| and the
        // cast of t / s into the half-precision level
        const int pa = acc_prec(L.prec);
        const double Nc = (double)points(h->dim, C.n);
        void *t = h->ws + C.off_t;
        RUN(h, st, "resid_restrict", l, N * 2 * sb(L.prec) + Nc * sb(pa),
            level_restrict(h, l, L.prec, pa, b, cbuf(h, l, h->cur[l]), t, st));
        RUN(h, st, "rescale_max", l + 1, Nc * sb(pa),
            launch_absmax(pa, t, (long)C.elems, at_ws<double>(h, h->off_rpart), rscal(h, l + 1), st));
        RUN(h, st, "rescale_cast", l + 1, Nc * (sb(pa) + sb(C.prec)),
            launch_scale_cast(pa, C.prec, t, rscal(h, l + 1), bbuf(h, l + 1), (long)C.elems, st));
        return hipSuccess;
    }
    RUN(h, st, "resid_restrict", l, bytes,
        level_restrict(h, l, L.prec, C.prec, b, cbuf(h, l, h->cur[l]), bbuf(h, l + 1), st));
    return hipSuccess;
}

hipError_t enq_coarse(mg_ctx *h, hipStream_t st, int l) {
    LevelPlan &L = h->lv[l];
    if (L.n > 1) {
        // CG on a base level of more than one point (Section 4.2)
        const long N = (long)points(h->dim, L.n);
        const int maxit = h->opt.base_max_iter > 0 ? h->opt.base_max_iter : (int)std::min<long>(10000, N);
        RUN(h, st, "cg_base", l, (double)N * 2 * sb(L.prec),
            launch_cg_base(h->dim, L.prec, L.n, L.P, bbuf(h, l), cbuf(h, l, 0), h->ws + L.off_cg,
                           cg_scratch_stride(L.prec, L.elems), h->opt.base_tol, maxit, h->q1 ? 1 : 0, st));
        h->cur[l] = 0;
        return hipSuccess;
    }
    RUN(h, st, "coarse_solve", l, 2 * sb(L.prec),
        h->q1 ? launch_q1_coarse(h->dim, L.prec, bbuf(h, l), cbuf(h, l, 0), st)
              : launch_coarse(h->dim, L.prec, bbuf(h, l), cbuf(h, l, 0), st));
    h->cur[l] = 0;
    return hipSuccess;
}

hipError_t enq_prolong(mg_ctx *h, hipStream_t st, int l, const void *b) {
    LevelPlan &L = h->lv[l], &C = h->lv[l + 1];
    const double N = (double)points(h->dim, L.n);
    const double bytes = N * 3 * sb(L.prec) + (double)points(h->dim, C.n) * sb(C.prec);
    const int cur = h->cur[l];
    if (C.rescale) {
        // the coarse correction times s, in the fine accumulator format
        const int pa = acc_prec(L.prec);
        const double Nc = (double)points(h->dim, C.n);
        void *t = h->ws + C.off_t;
        RUN(h, st, "rescale_widen", l + 1, Nc * (sb(C.prec) + sb(pa)),
            launch_scale_widen(C.prec, pa, cbuf(h, l + 1, h->cur[l + 1]), rscal(h, l + 1), t, (long)C.elems, st));
        RUN(h, st, "prolong_sweep", l, N * 3 * sb(L.prec) + Nc * sb(pa),
            level_prolong(h, l, L.prec, pa, cbuf(h, l, cur), t, b, cbuf(h, l, cur ^ 1), st));
        h->cur[l] = cur ^ 1;
        return hipSuccess;
    }
    RUN(h, st, "prolong_sweep", l, bytes,
        level_prolong(h, l, L.prec, C.prec, cbuf(h, l, cur), cbuf(h, l + 1, h->cur[l + 1]), b, cbuf(h, l, cur ^ 1),
                      st));
    h->cur[l] = cur ^ 1;
    return hipSuccess;
}

hipError_t enq_post(mg_ctx *h, hipStream_t st, int l, const void *b, bool skip_last = false) {
    LevelPlan &L = h->lv[l];
    const double N = (double)points(h->dim, L.n);
    for (int k = 1; k < h->opt.nu2 - (skip_last ? 1 : 0); ++k) {
        const int cur = h->cur[l];
        RUN(h, st, "sweep", l, N * 3 * sb(L.prec), level_sweep(h, l, L.prec, b, cbuf(h, l, cur), cbuf(h, l, cur ^ 1), st));
        h->cur[l] = cur ^ 1;
    }
    return hipSuccess;
}

// Finest-level right-hand side modes of a V-cycle.
enum RhsMode { RHS_B = 0, RHS_SCALED_R = 1, RHS_ALIAS_R = 2 };

// Pre-smoothing of level l and restriction of its residual to level l + 1.
// warm: the finest level continues from its current correction (a further
// V-cycle of the same refinement step) with nu1 plain sweeps.
hipError_t enq_vcycle_down(mg_ctx *h, hipStream_t st, RhsMode mode, int l, const void *rhs, bool warm = false) {
    hipError_t e;
    if (l == 0 && warm) {
        LevelPlan &L = h->lv[0];
        const double N = (double)points(h->dim, L.n);
        for (int k = 0; k < h->opt.nu1; ++k) {
            const int cur = h->cur[0];
            RUN(h, st, "sweep", 0, N * 3 * sb(L.prec), level_sweep(h, 0, L.prec, rhs, cbuf(h, 0, cur), cbuf(h, 0, cur ^ 1), st));
            h->cur[0] = cur ^ 1;
        }
        return enq_restrict(h, st, 0, rhs);
    }
    if (l >= 1 && h->lv[l].fsr) {
        LevelPlan &L = h->lv[l], &C = h->lv[l + 1];
        const double N = (double)points(h->dim, L.n);
        RUN(h, st, "smooth_restrict", l, N * 2 * sb(L.prec) + (double)points(h->dim, C.n) * sb(C.prec),
            launch_smooth_restrict_b(L.prec, C.prec, L.P, rhs, cbuf(h, l, 0), bbuf(h, l + 1), h->opt.omega, L.fsrsh,
                                     st));
        h->cur[l] = 0;
        return hipSuccess;
    }
    if (l == 0 && mode == RHS_SCALED_R && h->fused_sr) {
        LevelPlan &L = h->lv[0], &C = h->lv[1];
        const double N = (double)points(h->dim, L.n);
        RUN(h, st, "smooth_restrict", 0, N * (8 + 2 * sb(L.prec)) + (double)points(h->dim, C.n) * sb(C.prec),
            launch_smooth_restrict(L.prec, C.prec, L.P, Rbuf(h), scal(h), bbuf(h, 0), cbuf(h, 0, 0), bbuf(h, 1),
                                   h->opt.omega, h->srsh, st));
        h->cur[0] = 0;
        return hipSuccess;
    }
    if (l == 0 && mode == RHS_ALIAS_R && h->fused_sr) {
        LevelPlan &L = h->lv[0], &C = h->lv[1];
        const double N = (double)points(h->dim, L.n);
        RUN(h, st, "smooth_restrict", 0, N * 16 + (double)points(h->dim, C.n) * sb(C.prec),
            launch_smooth_restrict_b(P_F64, C.prec, L.P, Rbuf(h), cbuf(h, 0, 0), bbuf(h, 1), h->opt.omega, h->srsh,
                                     st));
        h->cur[0] = 0;
        return hipSuccess;
    }
    if (l == 0 && mode == RHS_ALIAS_R) {
        // FP64 baseline without scaling: the residual is the right-hand side
        LevelPlan &L = h->lv[0];
        const double N = (double)points(h->dim, L.n);
        const bool two = h->opt.nu1 >= 2 && !h->q1;
        RUN(h, st, two ? "smooth2" : "smooth1", 0, N * 16,
            level_first(h, 0, P_F64, Rbuf(h), nullptr, nullptr, nullptr, cbuf(h, 0, 0), two, st));
        int cur = 0;
        for (int k = two ? 2 : 1; k < h->opt.nu1; ++k) {
            RUN(h, st, "sweep", 0, N * 24, level_sweep(h, 0, P_F64, Rbuf(h), cbuf(h, 0, cur), cbuf(h, 0, cur ^ 1), st));
            cur ^= 1;
        }
        h->cur[0] = cur;
    } else {
        if ((e = enq_presmooth(h, st, l, l == 0 && mode == RHS_SCALED_R)) != hipSuccess) return e;
    }
    return enq_restrict(h, st, l, rhs);
}

// First level of the fused coarse end (see launch_tail), or nl - 1 when the
// V-cycle has none: the first level l >= 1 of pitch <= 16 (<= 8 for FP64)
// from which all levels above the base share one format and fit in LDS.
int tail_level(const mg_ctx *h) {
    const int nl = h->nl;
    if (!h->tail_on || h->dim != 3 || nl < 3 || h->lv[nl - 1].n > 1) return nl - 1;
    for (int l = 1; l < nl - 1; ++l) {
        const int P = h->lv[l].P, prec = h->lv[l].prec;
        if (P > (prec == P_F64 ? 8 : 16)) continue;
        bool same = true;
        for (int j = l; j < nl - 1; ++j) same = same && h->lv[j].prec == prec;
        // the fused coarse end has no rescaled restriction inside it
        for (int j = l + 1; j < nl; ++j) same = same && !h->lv[j].rescale;
        if (!same) continue;
        const size_t lds = tail_lds_bytes(prec, h->lv[nl - 1].prec, P, nl - 1 - l);
        if (lds > 0 && lds <= 65536) return l;
    }
    return nl - 1;
}

// One V-cycle.  warm: the finest level starts from its current correction;
// skip0: its last post-sweep is left to the fused sweep + update.
hipError_t enq_vcycle(mg_ctx *h, hipStream_t st, RhsMode mode, bool warm = false, bool skip0 = false) {
    const int nl = h->nl;
    const void *rhs[32];  // (levels are at most 13; no heap use on this path)
    for (int l = 0; l < nl; ++l) rhs[l] = bbuf(h, l);
    if (mode == RHS_ALIAS_R) rhs[0] = Rbuf(h);
    hipError_t e;
    const int lt = tail_level(h);
    if (lt < nl - 1) {
        // levels 0 .. lt-1 as separate launches, lt .. base fused
        for (int l = 0; l < lt; ++l) {
            if ((e = enq_vcycle_down(h, st, mode, l, rhs[l], warm)) != hipSuccess) return e;
        }
        const LevelPlan &T = h->lv[lt];
        RUN(h, st, "coarse_tail", lt, 0.0,
            launch_tail(T.prec, h->lv[nl - 1].prec, T.P, nl - 1 - lt, bbuf(h, lt), cbuf(h, lt, 0), h->opt.nu1,
                        h->opt.nu2, h->opt.omega, st));
        h->cur[lt] = 0;
        for (int l = lt - 1; l >= 0; --l) {
            if ((e = enq_prolong(h, st, l, rhs[l])) != hipSuccess) return e;
            if ((e = enq_post(h, st, l, rhs[l], l == 0 && skip0)) != hipSuccess) return e;
        }
        return hipSuccess;
    }
    for (int l = 0; l < nl - 1; ++l) {
        if ((e = enq_vcycle_down(h, st, mode, l, rhs[l], warm)) != hipSuccess) return e;
    }
    if ((e = enq_coarse(h, st, nl - 1)) != hipSuccess) return e;
    for (int l = nl - 2; l >= 0; --l) {
        if ((e = enq_prolong(h, st, l, rhs[l])) != hipSuccess) return e;
        if ((e = enq_post(h, st, l, rhs[l], l == 0 && skip0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

bool finest_alias(mg_ctx *h) { return h->lv[0].prec == P_F64 && !h->opt.residual_scaling; }

// The fused last sweep + update needs at least two post-sweeps.  It reads
// the stored right-hand side b, or (su_r) forms b = round(r / alpha) from the
// FP64 residual r, as the first smoothing did: s bytes per point fewer, but r
// is read on the tile's halo rows too.  With the FP64 map and no scaling r
// itself is the right-hand side, so that form is the only one.  A block then
// reads r on rows its neighbours update, so the new residual goes to a second
// array (swaps_r).
bool fusion_possible(mg_ctx *h) {
    return h->fuse_on && !h->batched && !h->nrhs && h->dim == 3 && h->nl >= 2 && h->opt.nu2 >= 2 &&
           (!h->su_r || h->off_R2) && (h->su_r || !finest_alias(h)) &&
           sweep_update_ok(h->lv[0].P, h->lv[0].prec, h->fsh);
}

// Whether a refinement step writes its residual to the other array.
bool swaps_r(const mg_ctx *h) { return h->fused && h->su_r; }

// Whether the step postpones the solution update (the fused finite-difference
// update, or the Q1 update).
bool defers(const mg_ctx *h) { return h->defer > 0 && (h->fused || h->q1); }

// The factor of the update u += alpha f c: h^2 for finite differences in
// grid-scaled units, h^(2-D) for the Q1 elements.
double update_factor(const mg_ctx *h) {
    const double hh = 1.0 / (double)(h->lv[0].n + 1);
    if (h->q1) return h->dim == 3 ? 1.0 / hh : 1.0;
    return hh * hh;
}

// Arguments of the fused sweep + update for the current state.
SweepUpdateArgs su_args(mg_ctx *h, const void *c) {
    const LevelPlan &L = h->lv[0];
    const double hh = 1.0 / (double)(L.n + 1);
    SweepUpdateArgs a;
    a.c = c;
    a.b = h->su_r ? (const void *)Rbuf(h) : bbuf(h, 0);  // b == R: b is formed from r
    a.R = Rbuf(h);
    a.Rout = h->su_r ? Rnext(h) : Rbuf(h);
    a.U = Ubuf(h);
    if (defers(h)) {
        a.cdefer = h->ws + h->off_cdef;
        a.ctr = at_ws<int>(h, h->off_dctr);
        a.cstride = h->cdef_stride;
        a.adef = at_ws<double>(h, h->off_adef);
    }
    a.scal = scal(h);
    a.h2 = hh * hh;
    a.omega = h->opt.omega;
    a.part = part(h);
    return a;
}

// The fused first smoothing + restriction replaces exactly two pre-sweeps
// of the scaled residual (or, for the FP64 map without scaling, of the
// residual itself) and the restriction of their result.
bool fusion_sr_possible(mg_ctx *h) {
    return h->fuse_sr_on && !h->batched && !h->nrhs && h->dim == 3 && h->nl >= 2 && h->opt.nu1 == 2 &&
           !h->lv[1].rescale && smooth_restrict_ok(h->lv[0].P, h->lv[0].prec, h->srsh);
}

void set_fused_sr(mg_ctx *h, bool on) { h->fused_sr = on && fusion_sr_possible(h); }

// The same fusion on a coarser level l (right-hand side b_l from memory).
bool fusion_srb_possible(mg_ctx *h, int l) {
    if (l < 1 || l + 1 >= h->nl) return false;
    const LevelPlan &L = h->lv[l];
    return L.fsr_on && !h->batched && !h->nrhs && h->dim == 3 && h->opt.nu1 == 2 &&
           !h->lv[l + 1].rescale && smooth_restrict_ok(L.P, L.prec, L.fsrsh);
}

void set_fused_srb(mg_ctx *h, int l, bool on) { h->lv[l].fsr = on && fusion_srb_possible(h, l); }

// A fused-kernel shape that fits level l: the most coarse rows per tile that
// the kernel allows, 16 coarse planes per chunk (fewer on small levels).
RShape default_srshape(const LevelPlan &L) {
    for (int tyc = 3; tyc >= 1; --tyc) {
        const RShape r{8, tyc, std::max(1, std::min(16, L.P / 2 - 1)), 3};
        if (smooth_restrict_ok(L.P, L.prec, r)) return r;
    }
    return RShape{8, 1, 1, 3};
}

void set_fused(mg_ctx *h, bool on) {
    h->fused = on && fusion_possible(h);
    const LevelPlan &L = h->lv[0];
    h->outer_parts = h->q1      ? q1_outer_blocks(h->dim, L.n, L.prec, L.q1s[2])
                     : h->fused ? sweep_update_blocks(L.P, h->fsh)
                                : stencil_blocks(h->dim, L.P, L.osh);
}

// One refinement step of Algorithm 2 (scale and cast, V-cycle, update) plus
// the norm readback.
// The V-cycle part of a refinement step (writes only level vectors).
// The V-cycles of one refinement step: the first from the scaled residual
// (or, for the FP64 baseline, the residual itself) and zero, each further one
// from the correction so far on the same right-hand side.  Inside a step the
// last finest-level sweep of the last cycle runs fused with the update.
hipError_t enq_cycle(mg_ctx *h, hipStream_t st) {
    const bool alias = finest_alias(h);
    const int m = std::max(1, h->opt.cycles_per_step);
    for (int j = 0; j < m; ++j) {
        const RhsMode mode = alias ? RHS_ALIAS_R : j == 0 ? RHS_SCALED_R : RHS_B;
        const hipError_t e = enq_vcycle(h, st, mode, j > 0, j == m - 1 && h->fused);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The update part: u, r, norms, alpha, and the norm readback (with the fused
// form, also the last post-smoothing sweep of the finest level).
hipError_t enq_update(mg_ctx *h, hipStream_t st) {
    LevelPlan &L = h->lv[0];
    const double hh = 1.0 / (double)(L.n + 1);
    const double N = (double)points(h->dim, L.n);
    if (h->fused) {
        // bytes: c, b, r read, r written, u read and written; b formed from
        // r is not read; a postponed update writes c' instead of reading and
        // writing u
        const double s = sb(L.prec);
        const double by = (h->su_r ? s + 16 : 2 * s + 16) + (defers(h) ? s : 16);
        RUN(h, st, defers(h) ? "sweep_update_defer" : "sweep_update", 0, N * by,
            launch_sweep_update(L.prec, L.P, su_args(h, cbuf(h, 0, h->cur[0])), h->fsh, st));
    } else if (h->q1) {
        // U += alpha h^(2-D) c, R -= alpha S c; postponed: c copied to the ring
        const bool d = defers(h);
        RUN(h, st, d ? "ir_update_defer" : "ir_update", 0, N * (d ? 16 + 2 * sb(L.prec) : 32 + sb(L.prec)),
            launch_q1_outer(h->dim, L.prec, L.n, L.P, cbuf(h, 0, h->cur[0]), Rbuf(h), Ubuf(h), scal(h),
                            update_factor(h), part(h), st, d ? (void *)(h->ws + h->off_cdef) : nullptr,
                            h->cdef_stride, d ? at_ws<double>(h, h->off_adef) : nullptr,
                            d ? at_ws<int>(h, h->off_dctr) : nullptr, L.q1s[2]));
    } else {
        RUN(h, st, "ir_update", 0, N * (32 + sb(L.prec)),
            launch_outer_update(h->dim, L.prec, L.P, cbuf(h, 0, h->cur[0]), Rbuf(h), Ubuf(h), scal(h), hh * hh,
                                part(h), L.osh, st));
    }
    RUN(h, st, "norm_finalize", 0, 16.0 * h->outer_parts,
        launch_finalize(part(h), h->outer_parts, scal(h), h->ascale, st,
                        defers(h) ? at_ws<int>(h, h->off_dctr) : nullptr));
    return hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st);
}

// Add the postponed corrections to u (their slots in order) and empty the
// ring; nothing to do without postponed corrections.
hipError_t enq_flush(mg_ctx *h, hipStream_t st) {
    const LevelPlan &L = h->lv[0];
    const bool zero = h->u_zero;  // the first flush of a solve from zero starts from 0 instead of reading u
    h->u_zero = false;
    if (h->pending == 0) return zero ? launch_fill_zero(Ubuf(h), align_up(L.elems * sizeof(double), 16), st) : hipSuccess;
    const int k = h->pending;
    h->pending = 0;
    RUN(h, st, "defer_flush", 0, (double)points(h->dim, L.n) * ((zero ? 8 : 16) + k * sb(L.prec)),
        launch_defer_flush(L.prec, h->ws + h->off_cdef, h->cdef_stride, at_ws<double>(h, h->off_adef), k,
                           update_factor(h), Ubuf(h), L.elems, at_ws<int>(h, h->off_dctr), st, zero));
    return hipSuccess;
}

// Host bookkeeping after a step's update has been queued: the residual array
// it wrote becomes current, and its correction waits in the ring (which is
// flushed when full).
hipError_t after_update(mg_ctx *h, hipStream_t st) {
    if (swaps_r(h)) h->rpar ^= 1;
    if (!defers(h)) return hipSuccess;
    ++h->pending;
    return h->pending >= h->defer ? enq_flush(h, st) : hipSuccess;
}

// One refinement step of Algorithm 2 (scale and cast, V-cycle, update) plus
// the norm readback.
hipError_t enq_step(mg_ctx *h, hipStream_t st) {
    hipError_t e = enq_cycle(h, st);
    return e != hipSuccess ? e : enq_update(h, st);
}

void drop_graph(mg_ctx *h) {
    for (hipGraphExec_t *x : {&h->gexec, &h->gexec2, &h->gexec_p1, &h->gexec2_p1}) {
        if (*x) (void)hipGraphExecDestroy(*x);
        *x = nullptr;
    }
    for (hipGraph_t *g : {&h->graph, &h->graph2, &h->graph_p1, &h->graph2_p1}) {
        if (*g) (void)hipGraphDestroy(*g);
        *g = nullptr;
    }
}

// Capture the cycle part and the update part of a refinement step as two
// graphs, so that the next cycle can be queued before the host has read the
// current step's norm.  When steps swap the residual arrays, a second pair is
// captured for steps that start from the second array.
mg_status_t ensure_graph(mg_ctx *h) {
    const bool two = swaps_r(h);
    if (h->gexec && h->gexec2 && (!two || (h->gexec_p1 && h->gexec2_p1))) return MG_OK;
    drop_graph(h);
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    const int keep = h->rpar;
    for (int par = 0; par < (two ? 2 : 1); ++par) {
        h->rpar = par;
        for (int part = 0; part < 2; ++part) {
            HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = part == 0 ? enq_cycle(h, h->cap_stream) : enq_update(h, h->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
            if (e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                h->rpar = keep;
                return fail(MG_ERR_HIP, "capture of the refinement step failed: %s", hipGetErrorString(e));
            }
            if (e2 != hipSuccess) {
                h->rpar = keep;
                return fail(MG_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
            }
            hipGraph_t &gs = par == 0 ? (part == 0 ? h->graph : h->graph2) : (part == 0 ? h->graph_p1 : h->graph2_p1);
            hipGraphExec_t &gx =
                par == 0 ? (part == 0 ? h->gexec : h->gexec2) : (part == 0 ? h->gexec_p1 : h->gexec2_p1);
            gs = g;
            const hipError_t e3 = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
            if (e3 != hipSuccess) {
                h->rpar = keep;
                return fail(MG_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
            }
        }
    }
    h->rpar = keep;
    return MG_OK;
}

void build_batched_plan(mg_ctx *h, char *base);
hipError_t enq_batched_step(mg_ctx *h, hipStream_t st);
hipError_t enq_multi_step(mg_ctx *h, hipStream_t st);
mg_status_t autotune_batched(mg_ctx *h, hipStream_t st);
mg_status_t autotune_multi(mg_ctx *h, hipStream_t st);
mg_status_t batched_upload(mg_ctx *h);

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
    if (s.dp < 1 || s.dp > 2 || (s.dp == 2 && s.ty == 0) || (s.sg != 0 && s.sg != 1)) return false;
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
    if (r.pipe < 0 || r.pipe > 4) return false;
    if (r.pipe >= 2 && (L.P / r.V > 64 || r.V < 4)) return false;  // rows must not straddle waves
    if (r.tyc < 1 || r.tyc > std::max(1, Pc - 1)) return false;
    const int G = h->dim == 3 ? 2 * r.tyc + 1 + (r.pipe ? 2 : 0) : 1;
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

// prolong: the prolongation family, which also tries reading its coarse rows
// from memory on the LDS-plane kernel (sg = 0)
std::vector<Shape> stencil_candidates(const mg_ctx *h, const LevelPlan &L, bool update, bool prolong = false) {
    std::vector<Shape> out;
    const int tys[] = {0, 2, 4, 6, 10, 14};
    const int zcs[] = {2, 4, 8, 16, 32, 64};
    for (int V : {4, 8})
        for (int ty : tys)
            for (int zc : zcs) {
                for (int dp = 1; dp <= (ty > 0 ? 2 : 1); ++dp) {
                    for (int sg = 1; sg >= (prolong && ty > 0 ? 0 : 1); --sg) {
                    Shape s{V, zc, 256, 1, ty, dp, sg};
                    if (ty == 0 && h->dim == 3 && zc < 8) continue;
                    if (update && V == 8 && ty > 0) continue;  // FP64 rows spill at V = 8
                    if (L.prec == P_F64 && V == 8 && ty > 0) continue;
                    if (stencil_ok(h, L, s)) out.push_back(s);
                    }
                }
            }
    return out;
}

// ---- persisted tuning -------------------------------------------------------
// With MGIR_TUNE_CACHE naming a file, the shapes the autotuner picked are
// appended to it as one line per configuration, and a later mg_bind_workspace
// with the same configuration on the same kind of device reads them back
// instead of timing again.  The key holds everything the choice depends on:
// device architecture and CU count, the library's tuning version, dimension,
// grid, level formats and the options that change the kernels.
constexpr int kTuneVersion = 4;

// The device part of a key: tuning version, architecture, CU count ("" when
// no device is current).
std::string device_key() {
    int dev = 0, cus = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    char buf[256];
    std::snprintf(buf, sizeof buf, "v%d|%s|cu%d", kTuneVersion, prop.gcnArchName, cus);
    return std::string(buf);
}

std::string tune_key(const mg_ctx *h) {
    const std::string dk = device_key();
    if (dk.empty()) return dk;
    char buf[512];
    int k = std::snprintf(buf, sizeof buf, "%s|d%d|n%d|L%d|nu%d,%d|sc%d|df%d|rh%d|cy%d|p", dk.c_str(), h->dim, h->n,
                          h->nl, h->opt.nu1, h->opt.nu2, h->opt.residual_scaling, h->opt.defer_update,
                          h->opt.rescale_half, h->opt.cycles_per_step);
    for (int l = 0; l < h->nl && k < (int)sizeof buf - 4; ++l) k += std::snprintf(buf + k, sizeof buf - k, "%d", h->lv[l].prec);
    return std::string(buf);
}

// The integers stored under key in the MGIR_TUNE_CACHE file (false: none).
bool cache_read(const std::string &key, std::vector<int> &v) {
    const char *path = std::getenv("MGIR_TUNE_CACHE");
    if (!path || !*path || key.empty()) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    std::string line;
    bool found = false;
    char chunk[4096];
    while (!found && std::fgets(chunk, sizeof chunk, f)) {
        line += chunk;
        if (line.empty() || line.back() != '\n') continue;  // a line longer than the chunk
        const size_t tab = line.find('\t');
        if (tab != std::string::npos && line.compare(0, tab, key) == 0 && tab == key.size()) {
            v.clear();
            const char *p = line.c_str() + tab + 1;
            for (;;) {
                char *end = nullptr;
                const long x = std::strtol(p, &end, 10);
                if (end == p) break;
                v.push_back((int)x);
                p = end;
            }
            found = true;
        }
        line.clear();
    }
    std::fclose(f);
    return found;
}

void cache_write(const std::string &key, const std::vector<int> &v) {
    const char *path = std::getenv("MGIR_TUNE_CACHE");
    if (!path || !*path || key.empty()) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s\t", key.c_str());
    for (size_t i = 0; i < v.size(); ++i) std::fprintf(f, i ? " %d" : "%d", v[i]);
    std::fprintf(f, "\n");
    std::fclose(f);
}

// The tuned state as integers: per level the three stencil shapes, the
// update shape, the restriction shape and the coarse fused form; then the
// finest-level fused forms.
void tune_state(const mg_ctx *h, std::vector<int> &v) {
    auto sh = [&](const Shape &s) { v.insert(v.end(), {s.V, s.zc, s.bs, s.xcd, s.ty, s.dp, s.sg}); };
    auto rs = [&](const RShape &r) { v.insert(v.end(), {r.V, r.tyc, r.zcc, r.pipe}); };
    for (int l = 0; l + 1 < h->nl; ++l) {
        const LevelPlan &L = h->lv[l];
        for (int f = 0; f < 3; ++f) sh(L.shs[f]);
        sh(L.osh);
        rs(L.rsh);
        rs(L.fsrsh);
        v.push_back(L.fsr ? 1 : 0);
    }
    rs(h->srsh);
    v.push_back(h->fused_sr ? 1 : 0);
    sh(h->fsh);
    v.push_back(h->fused ? 1 : 0);
    v.push_back(h->su_r ? 1 : 0);
}

// Apply a state read from the cache; false (and nothing changed) when any
// shape is not valid for this handle.
bool apply_tune_state(mg_ctx *h, const std::vector<int> &v) {
    const size_t per = 4 * 7 + 4 + 4 + 1, need = per * (h->nl - 1) + 4 + 1 + 7 + 1 + 1;
    if (v.size() != need) return false;
    size_t i = 0;
    auto sh = [&]() {
        Shape s{v[i], v[i + 1], v[i + 2], v[i + 3], v[i + 4], v[i + 5], v[i + 6]};
        i += 7;
        return s;
    };
    auto rs = [&]() { RShape r{v[i], v[i + 1], v[i + 2], v[i + 3]}; i += 4; return r; };
    std::vector<LevelPlan> lv = h->lv;
    std::vector<bool> fsr(h->nl, false);
    for (int l = 0; l + 1 < h->nl; ++l) {
        LevelPlan &L = lv[l];
        for (int f = 0; f < 3; ++f) {
            L.shs[f] = sh();
            if (!stencil_ok(h, L, L.shs[f])) return false;
        }
        L.osh = sh();
        if (l == 0 && (!stencil_ok(h, L, L.osh) || stencil_blocks(h->dim, L.P, L.osh) > h->max_parts)) return false;
        L.rsh = rs();
        if (!restrict_ok(h, L, L.rsh)) return false;
        L.fsrsh = rs();
        fsr[l] = v[i++] != 0;
    }
    const RShape srsh = rs();
    const bool fused_sr = v[i++] != 0;
    const Shape fsh = sh();
    const bool fused = v[i++] != 0;
    const bool su_r = v[i++] != 0;
    if (!su_r && finest_alias(h)) return false;
    h->lv = lv;
    for (int l = 1; l + 1 < h->nl; ++l) set_fused_srb(h, l, fsr[l]);
    h->srsh = srsh;
    set_fused_sr(h, fused_sr);
    h->fsh = fsh;
    h->su_r = su_r;
    set_fused(h, fused);
    return true;
}

bool tune_cache_load(mg_ctx *h, const std::string &key) {
    std::vector<int> v;
    return cache_read(key, v) && apply_tune_state(h, v);
}

void tune_cache_store(const mg_ctx *h, const std::string &key) {
    std::vector<int> v;
    tune_state(h, v);
    cache_write(key, v);
}

mg_status_t autotune_timed(mg_ctx *h, hipStream_t st);

mg_status_t autotune(mg_ctx *h, hipStream_t st) {
    const std::string key = tune_key(h);
    if (tune_cache_load(h, key)) return MG_OK;
    const mg_status_t s = autotune_timed(h, st);
    if (s == MG_OK) tune_cache_store(h, key);
    return s;
}

mg_status_t autotune_timed(mg_ctx *h, hipStream_t st) {
    const int D = h->dim;
    for (int l = 0; l + 1 < h->nl; ++l) {
        LevelPlan &L = h->lv[l];
        if (L.P < 8) continue;
        // each smoothing-family kernel separately; on the finest level the
        // first pre-smoothing is timed in the form the refinement loop uses
        const bool scaled0 = l == 0 && !finest_alias(h);
        const void *b0 = (l == 0 && finest_alias(h)) ? (const void *)Rbuf(h) : bbuf(h, l);
        float fam_best[3] = {0.f, 0.f, 0.f};
        for (int fam = 0; fam < 3; ++fam) {
            float best = 1e30f;
            Shape bs = L.shs[fam];
            for (const Shape &s : stencil_candidates(h, L, false, fam == SH_PROLONG)) {
                const float t = time_ms(st, [&]() -> hipError_t {
                    if (fam == SH_SMOOTH)
                        return scaled0 ? launch_smooth_first(D, L.prec, L.P, nullptr, Rbuf(h), scal(h), bbuf(h, l),
                                                             cbuf(h, l, 0), h->opt.omega, true, s, st)
                                       : launch_smooth_first(D, L.prec, L.P, b0, nullptr, nullptr, nullptr,
                                                             cbuf(h, l, 0), h->opt.omega, true, s, st);
                    if (fam == SH_SWEEP)
                        return launch_sweep(D, L.prec, L.P, b0, cbuf(h, l, 0), cbuf(h, l, 1), h->opt.omega, s, st);
                    return launch_prolong(D, L.prec, h->lv[l + 1].prec, L.P, cbuf(h, l, 1), cbuf(h, l + 1, 0), b0,
                                          cbuf(h, l, 0), h->opt.omega, true, s, st);
                }, 3);
                if (t < best) best = t, bs = s;
            }
            L.shs[fam] = bs;
            fam_best[fam] = best;
        }
        // residual + restriction
        float best = 1e30f;
        RShape br = L.rsh;
        for (int V : {4, 8})
            for (int tyc : {1, 2, 3, 4, 5, 7})
                for (int zcc : {2, 4, 8, 16, 32})
                    for (int pipe : {0, 1, 2, 3, 4}) {
                    RShape r{V, tyc, zcc, pipe};
                    if (!restrict_ok(h, L, r)) continue;
                    const float t = time_ms(st, [&]() {
                        return launch_restrict(D, L.prec, h->lv[l + 1].prec, L.P, bbuf(h, l), cbuf(h, l, 0),
                                               bbuf(h, l + 1), r, st);
                    }, 3);
                    if (t < best) best = t, br = r;
                }
        L.rsh = br;
        if (l == 0 ? fusion_sr_possible(h) : fusion_srb_possible(h, l)) {
            // the fused first smoothing + restriction against the two kernels
            float bf = 1e30f;
            RShape bsr = l == 0 ? h->srsh : L.fsrsh;
            int dev = 0, cus = 256;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            for (int tyc : {1, 2, 3}) {
                // powers of two, and the shortest chunk for each chunk count
                // whose block count nearly fills up to six whole rounds of one
                // block per CU
                std::vector<int> zs{4, 8, 16, 32};
                const int Pc = L.P / 2, ytiles = (Pc - 1 + tyc - 1) / tyc;
                int last_chunks = 0;
                for (int zcc = 6; zcc <= Pc - 1; ++zcc) {
                    const int chunks = (Pc - 1 + zcc - 1) / zcc;
                    if (chunks == last_chunks) continue;
                    last_chunks = chunks;
                    const long nb = (long)ytiles * chunks;
                    const long rounds = (nb + cus - 1) / cus;
                    if (rounds <= 6 && nb >= 0.97 * rounds * cus && std::find(zs.begin(), zs.end(), zcc) == zs.end())
                        zs.push_back(zcc);
                }
                for (int zcc : zs)
                    for (int lw : {3, 4}) {  // c1, c2 in LDS in FP32/FP64, or in the 2-byte format
                    const RShape r{8, tyc, zcc, lw};
                    if (!smooth_restrict_ok(L.P, L.prec, r)) continue;
                    const float t = time_ms(st, [&]() {
                        if (l == 0 && finest_alias(h))
                            return launch_smooth_restrict_b(L.prec, h->lv[1].prec, L.P, Rbuf(h), cbuf(h, 0, 0),
                                                            bbuf(h, 1), h->opt.omega, r, st);
                        if (l == 0)
                            return launch_smooth_restrict(L.prec, h->lv[1].prec, L.P, Rbuf(h), scal(h), bbuf(h, 0),
                                                          cbuf(h, 0, 0), bbuf(h, 1), h->opt.omega, r, st);
                        return launch_smooth_restrict_b(L.prec, h->lv[l + 1].prec, L.P, bbuf(h, l), cbuf(h, l, 0),
                                                        bbuf(h, l + 1), h->opt.omega, r, st);
                    }, 3);
                    if (t < bf) bf = t, bsr = r;
                }
            }
            const bool win = bf < best + fam_best[SH_SMOOTH];
            if (l == 0) {
                h->srsh = bsr;
                set_fused_sr(h, win);
            } else {
                L.fsrsh = bsr;
                set_fused_srb(h, l, win);
            }
        }
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
            // the fused last sweep + update against the two kernels it replaces
            // (both ways of getting the right-hand side where both apply)
            if (fusion_possible(h)) {
                float bf = 1e30f;
                Shape bsu = h->fsh;
                bool bsr = h->su_r;
                const bool keep_r = h->su_r;
                for (int from_r = finest_alias(h) ? 1 : 0; from_r <= 1; ++from_r)
                    for (int ty : {1, 2, 3, 4})
                        for (int zc : {4, 8, 16, 32, 64}) {
                            const Shape s{4, zc, 256, 1, ty};
                            if (!sweep_update_ok(L.P, L.prec, s)) continue;
                            const bool was = h->fused;
                            h->fused = true;  // the arguments of the form the step would use
                            h->su_r = from_r != 0;
                            const SweepUpdateArgs q = su_args(h, cbuf(h, 0, 0));
                            h->fused = was;
                            h->su_r = keep_r;
                            const float t =
                                time_ms(st, [&]() { return launch_sweep_update(L.prec, L.P, q, s, st); }, 3);
                            if (t < bf) bf = t, bsu = s, bsr = from_r != 0;
                        }
                h->fsh = bsu;
                h->su_r = bsr;
                set_fused(h, bf < best + fam_best[SH_SWEEP]);
            }
        }
    }
    HIPCHK(hipMemsetAsync(h->ws, 0, h->ws_need, st));
    HIPCHK(hipStreamSynchronize(st));
    return MG_OK;
}

// Q1 handles: which of a level's LDS-staged kernels a shape kind names (0 the
// sweep, 1 the residual ahead of the restriction, 2 the update; -1 none).
int q1_kind(int kind) {
    return kind == MG_SHAPE_SWEEP ? 0 : kind == MG_SHAPE_RESTRICT ? 1 : kind == MG_SHAPE_UPDATE ? 2 : -1;
}

// The Q1 shapes as integers: per level {ty, zc, split} of the sweep, the
// residual and the update.
bool apply_q1_state(mg_ctx *h, const std::vector<int> &v) {
    if (v.size() != (size_t)9 * (h->nl - 1)) return false;
    std::vector<LevelPlan> lv = h->lv;
    for (int l = 0; l + 1 < h->nl; ++l)
        for (int k = 0; k < 3; ++k) {
            const int *e = &v[9 * l + 3 * k];
            const Q1Shape q{e[0], e[1], e[2]};
            if (!q1_shape_ok(h->dim, lv[l].prec, lv[l].n, lv[l].P, k, q) || (k == 2 && l > 0 && q.ty != 0))
                return false;
            lv[l].q1s[k] = q;
        }
    h->lv = lv;
    set_fused(h, h->fused);  // the update's partial count
    return true;
}

// The Q1 autotuner: on each level that takes the LDS-staged kernels, each of
// them timed over {ty, zc} (the residual also as two kernels, split = 1)
// against the built-in shape, which stays unless another is faster.  The
// result is cached like the finite-difference one.
mg_status_t autotune_q1(mg_ctx *h, hipStream_t st) {
    const std::string key = tune_key(h).empty() ? std::string() : tune_key(h) + "|q1";
    std::vector<int> v;
    if (cache_read(key, v) && apply_q1_state(h, v)) return MG_OK;
    const int D = h->dim;
    for (int l = 0; l + 1 < h->nl; ++l) {
        LevelPlan &L = h->lv[l];
        if (!q1_lds_level(D, L.prec, L.n, L.P)) continue;
        for (int k = 0; k < (l == 0 ? 3 : 2); ++k) {
            auto run = [&](const Q1Shape &q) -> hipError_t {
                if (k == 0)
                    return launch_q1_sweep(D, L.prec, L.n, L.P, bbuf(h, l), cbuf(h, l, 0), cbuf(h, l, 1), h->opt.omega,
                                           st, q);
                if (k == 1)
                    return launch_q1_restrict(D, L.prec, h->lv[l + 1].prec, L.n, L.P, bbuf(h, l), cbuf(h, l, 0),
                                              h->ws + h->off_q1r, bbuf(h, l + 1), st, q);
                const bool d = h->defer > 0;  // the ring counter is zero: slot 0
                return launch_q1_outer(D, L.prec, L.n, L.P, cbuf(h, 0, 0), Rbuf(h), Ubuf(h), scal(h),
                                       update_factor(h), part(h), st, d ? (void *)(h->ws + h->off_cdef) : nullptr,
                                       h->cdef_stride, d ? at_ws<double>(h, h->off_adef) : nullptr,
                                       d ? at_ws<int>(h, h->off_dctr) : nullptr, q);
            };
            Q1Shape best{};
            float tb = time_ms(st, [&]() { return run(Q1Shape{}); }, 5);
            for (int split = 0; split <= (k == 1 ? 1 : 0); ++split)
                for (int ty = split ? 0 : 1; ty <= 8; ++ty)
                    for (int zc : {0, 2, 4, 8, 16, 32}) {
                        const Q1Shape q{ty, zc, split};
                        if ((ty == 0) != (zc == 0) || (ty == 0 && !split)) continue;
                        if (!q1_shape_ok(D, L.prec, L.n, L.P, k, q)) continue;
                        const float t = time_ms(st, [&]() { return run(q); }, 5);
                        if (t < tb) tb = t, best = q;
                    }
            L.q1s[k] = best;
        }
    }
    set_fused(h, h->fused);
    HIPCHK(hipMemsetAsync(h->ws, 0, h->ws_need, st));
    HIPCHK(hipStreamSynchronize(st));
    v.clear();
    for (int l = 0; l + 1 < h->nl; ++l)
        for (int k = 0; k < 3; ++k) v.insert(v.end(), {h->lv[l].q1s[k].ty, h->lv[l].q1s[k].zc, h->lv[l].q1s[k].split});
    cache_write(key, v);
    return MG_OK;
}
}  // namespace

namespace {
// The stencil-family or restriction shape of one level, as mg_get_shape returns it.
mg_status_t level_shape(const LevelPlan &L, int level, int kind, int *p, int np) {
    const bool stencil_kind = kind == MG_SHAPE_STENCIL || kind == MG_SHAPE_SMOOTH || kind == MG_SHAPE_SWEEP ||
                              kind == MG_SHAPE_PROLONG || (kind == MG_SHAPE_UPDATE && level == 0);
    if (stencil_kind && np >= 5) {
        const Shape &S = kind == MG_SHAPE_UPDATE   ? L.osh
                         : kind == MG_SHAPE_SMOOTH  ? L.shs[SH_SMOOTH]
                         : kind == MG_SHAPE_PROLONG ? L.shs[SH_PROLONG]
                                                    : L.shs[SH_SWEEP];
        p[0] = S.V, p[1] = S.zc, p[2] = S.bs, p[3] = S.xcd, p[4] = S.ty;
        if (np >= 6) p[5] = S.dp;
        if (np >= 7) p[6] = S.sg;
    } else if (kind == MG_SHAPE_RESTRICT && np >= 4) {
        p[0] = L.rsh.V, p[1] = L.rsh.tyc, p[2] = L.rsh.zcc, p[3] = L.rsh.pipe;
    } else {
        return fail(MG_ERR_ARG, "bad kind or too few values");
    }
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
    o->rescale_half = 0;
    o->cycles_per_step = 1;
    o->base_tol = 1e-4;
    o->base_max_iter = 0;
    o->discretization = MG_DISC_FD;
    o->defer_update = 0;
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
    mg_options_t o;
    mg_default_options(&o);
    if (opt) o = *opt;
    if (o.discretization != MG_DISC_FD && o.discretization != MG_DISC_Q1)
        return fail(MG_ERR_ARG, "discretization must be MG_DISC_FD or MG_DISC_Q1, got %d", o.discretization);
    const bool q1 = o.discretization == MG_DISC_Q1;
    if (q1) {
        if (n < 3 || n % 2 == 0 || n > 8191)
            return fail(MG_ERR_SHAPE, "Q1: n must be odd with 3 <= n <= 8191, got %d", n);
    } else if (n < 3 || ((n + 1) & n) != 0 || n > 4095) {
        return fail(MG_ERR_SHAPE, "n must be 2^m - 1 with 2 <= m <= 12, got %d", n);
    }
    if (dim == 3 && n > 1023)
        return fail(MG_ERR_SHAPE, "3-D grids are limited to n <= 1023 (one block must hold three fine rows)");
    // levels of the full hierarchy: halve while the size is odd and above one
    int m = 1;
    for (int t = n; t > 1 && t % 2 == 1; t = (t - 1) / 2) ++m;
    if (nlevels != 0 && (nlevels < 2 || nlevels > m))
        return fail(MG_ERR_ARG, "nlevels must be 0 (the full hierarchy, %d levels) or 2..%d, got %d", m, m, nlevels);
    if (nlevels) m = nlevels;  // from here on m counts the levels used
    {
        int nb = n;
        for (int l = 1; l < m; ++l) nb = (nb - 1) / 2;
        if (points(dim, nb) > kMaxBasePoints)
            return fail(MG_ERR_SHAPE, "base level of %d^%d points exceeds the %ld points of the one-workgroup CG; "
                        "use more levels", nb, dim, (long)kMaxBasePoints);
    }
    if (!(o.base_tol >= 0.0) || o.base_max_iter < 0)
        return fail(MG_ERR_ARG, "base_tol must be >= 0 and base_max_iter >= 0");
    if (o.nu1 < 1 || o.nu1 > 16 || o.nu2 < 1 || o.nu2 > 16)
        return fail(MG_ERR_ARG, "nu1 and nu2 must be in 1..16 (got %d, %d)", o.nu1, o.nu2);
    if (!(o.omega > 0.0 && o.omega < 2.0)) return fail(MG_ERR_ARG, "omega must be in (0, 2)");
    if (o.max_iter < 0) return fail(MG_ERR_ARG, "max_iter must be >= 0");
    if (!(o.rtol >= 0.0)) return fail(MG_ERR_ARG, "rtol must be >= 0");
    if (o.cycles_per_step < 1 || o.cycles_per_step > 16)
        return fail(MG_ERR_ARG, "cycles_per_step must be in 1..16 (got %d)", o.cycles_per_step);
    if (o.defer_update < 0 || o.defer_update > kMaxDefer)
        return fail(MG_ERR_ARG, "defer_update must be in 0..%d (got %d)", kMaxDefer, o.defer_update);
    std::vector<int> prec(m, P_F64);
    if (level_prec)
        for (int i = 0; i < m; ++i) {
            if (!valid_prec((int)level_prec[i])) return fail(MG_ERR_PREC, "level_prec[%d] = %d is not a format", i, (int)level_prec[i]);
            prec[i] = (int)level_prec[i];
        }
    int ascale = 0;
    {
        std::vector<int> ns(m);
        std::vector<bool> resc(m, false);
        for (int l = 0, nn = n; l < m; ++l, nn = (nn - 1) / 2) {
            ns[l] = nn;
            resc[l] = o.rescale_half && l >= 1 && half_prec(prec[l]);
        }
        if (!alpha_code(dim, ns, prec, resc, o.residual_scaling, &ascale))
            return fail(MG_ERR_PREC, "an FP16 level entered by a rescaled restriction would exceed FP16's range "
                        "(its correction bound %.0f > %.0f): store it in BF16, FP32 or FP64",
                        correction_bound(dim, ns[1]), kHalfCorrectionBound);
    }
    mg_ctx *h = new mg_ctx();
    h->dim = dim;
    h->n = n;
    h->nl = m;
    h->opt = o;
    h->ascale = ascale;
    h->q1 = q1;
    if (q1) h->tail_on = h->fuse_on = h->fuse_sr_on = false;
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
        // (launch shapes of the finite-difference kernels; the Q1 kernels have
        // none, but the finest level's sizes the reduction partials)
        if (nn > 1 && (!q1 || l == 0)) {
            L.shs[SH_SMOOTH] = L.shs[SH_SWEEP] = L.shs[SH_PROLONG] = pick_shape(dim, L.P, L.prec);
            L.osh = pick_shape(dim, L.P, P_F64);  // FP64 rows dominate the update's registers
            L.rsh = pick_rshape(dim, L.P, L.prec);
        }
        nn = (nn - 1) / 2;
    }
    if (h->lv[m - 1].n > 1) {
        LevelPlan &B = h->lv[m - 1];
        B.off_cg = off;
        off += 4 * cg_scratch_stride(B.prec, B.elems);
    }
    if (q1) {
        size_t rb = 0;
        for (int l = 0; l + 1 < m; ++l) rb = std::max(rb, q1_resid_bytes(dim, h->lv[l].prec, h->lv[l].P));
        h->off_q1r = off;
        off += align_up(rb, 256);
    }
    if (o.rescale_half) {
        for (int l = 1; l < m; ++l) {
            LevelPlan &C = h->lv[l];
            if (!half_prec(C.prec)) continue;
            C.rescale = true;
            C.off_t = off;
            off += align_up(C.elems * prec_bytes(acc_prec(h->lv[l - 1].prec)), 256);
        }
        h->off_rs = off;
        off += align_up((size_t)2 * m * sizeof(double), 256);
        h->off_rpart = off;
        off += align_up(rescale_part_count() * sizeof(double), 256);
    }
    // everything a V-cycle on its own touches lies below this offset
    h->vc_bytes = off;
    const size_t fin = align_up(h->lv[0].elems * sizeof(double), 256);
    h->off_R = off;
    off += fin;
    h->off_U = off;
    off += fin;
    // the forms of the fused finest-level update (3-D finite differences)
    const bool fusable = dim == 3 && !q1 && m >= 2;
    if (fusable) {
        // the fused update that forms its right-hand side from r writes the
        // new residual to a second array (FP16/BF16 maps default to reading b)
        h->su_r = prec_bytes(prec[0]) >= 4;
        h->off_R2 = off;
        off += fin;
    }
    if ((fusable || q1) && o.defer_update > 0) {
        const LevelPlan &L = h->lv[0];
        h->defer = o.defer_update;
        h->cdef_stride = align_up(L.elems * prec_bytes(L.prec), 256) / prec_bytes(L.prec);
        h->off_cdef = off;
        off += (size_t)h->defer * h->cdef_stride * prec_bytes(L.prec);
        h->off_adef = off;
        off += align_up((size_t)h->defer * sizeof(double), 256);
        h->off_dctr = off;
        off += 256;
    }
    if (m > 1) {
        h->outer_parts = stencil_blocks(dim, h->lv[0].P, h->lv[0].osh);
        // room for the partials of any legal shape: V = 4, zc = 1, 64-thread
        // blocks (more than the fused kernel's one row per block, zc = 1)
        const int P0 = h->lv[0].P;
        const long worst = ((long)(P0 / 4) * (dim == 3 ? P0 : 1) * (P0 - 1) + 63) / 64;
        const long worst_fused = (long)(P0 - 1) * (P0 - 1);
        maxp = (int)std::max<long>(std::max<long>(h->outer_parts, worst), worst_fused);
        // the most rows per block the fused update allows (fewer for FP64 rows)
        for (int ty = std::max(1, std::min(4, P0 - 1)); ty >= 1; --ty) {
            h->fsh = Shape{4, std::max(1, std::min(16, P0 - 1)), 256, 1, ty};
            if (sweep_update_ok(P0, prec[0], h->fsh)) break;
        }
    }
    maxp = std::max(maxp, flat_blocks(points(dim, n)));
    h->max_parts = maxp;
    h->off_part = off;
    off += align_up((size_t)maxp * 2 * sizeof(double), 256);
    h->off_scal = off;
    off += 256;
    h->ws_need = off;
    if (m > 1) {
        // the fused update's FP64 rows need more than 64 KB of LDS at P = 512
        if (h->dim == 3 && sweep_update_prepare() != hipSuccess) h->fuse_on = false;
        set_fused(h, true);
        // the fused first smoothing + restriction needs more than 64 KB of LDS
        // for its larger tiles; without that permission it stays off
        if (h->dim != 3 || smooth_restrict_prepare() != hipSuccess) h->fuse_sr_on = false;
        h->srsh = default_srshape(h->lv[0]);
        set_fused_sr(h, true);
        // on the coarser levels (fewer tiles than CUs, often) the fused form
        // is usually slower than the two kernels: off unless the autotuner
        // finds it faster
        for (int l = 1; l + 1 < m; ++l) {
            h->lv[l].fsrsh = default_srshape(h->lv[l]);
            set_fused_srb(h, l, false);
        }
    }
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
    if (h->nrhs) {
        const int K = h->nrhs;
        if (!h->host_mask) HIPCHK(hipHostMalloc((void **)&h->host_mask, 2 * sizeof(int) * K, hipHostMallocDefault));
        if (!h->host_scal_m) HIPCHK(hipHostMalloc((void **)&h->host_scal_m, 4 * sizeof(double) * K, hipHostMallocDefault));
        if (h->opt.autotune) return autotune_multi(h, st);
        return MG_OK;
    }
    if (h->batched) {
        const int ni = (int)h->inst.size();
        if (!h->host_active) HIPCHK(hipHostMalloc((void **)&h->host_active, sizeof(int) * ni, hipHostMallocDefault));
        if (!h->host_scal_all)
            HIPCHK(hipHostMalloc((void **)&h->host_scal_all, 4 * sizeof(double) * ni, hipHostMallocDefault));
        if (h->opt.autotune) return autotune_batched(h, st);
        return batched_upload(h);
    }
    if (h->opt.autotune) {
        mg_status_t s = h->q1 ? autotune_q1(h, st) : autotune(h, st);
        if (s != MG_OK) return s;
    }
    return MG_OK;
}

mg_status_t mg_destroy(mg_handle h) {
    if (!h) return MG_OK;
    drop_graph(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->ev_norm) (void)hipEventDestroy(h->ev_norm);
    if (h->host_scal) (void)hipHostFree(h->host_scal);
    if (h->host_active) (void)hipHostFree(h->host_active);
    if (h->host_scal_all) (void)hipHostFree(h->host_scal_all);
    if (h->host_mask) (void)hipHostFree(h->host_mask);
    if (h->host_scal_m) (void)hipHostFree(h->host_scal_m);
    delete h;
    return MG_OK;
}

mg_status_t mg_alpha_shift(mg_handle h, int instance, int *shift) {
    if (!h || !shift) return fail(MG_ERR_ARG, "null argument");
    const int ni = h->batched ? (int)h->inst.size() : 1;
    if (instance < 0 || instance >= ni) return fail(MG_ERR_ARG, "instance %d out of range 0..%d", instance, ni - 1);
    const int code = h->batched ? h->inst[instance].ascale : h->ascale;
    *shift = code - 1;
    return MG_OK;
}

mg_status_t mg_levels(mg_handle h, int *nlevels) {
    if (!h || !nlevels) return fail(MG_ERR_ARG, "null argument");
    *nlevels = h->nl;
    return MG_OK;
}

mg_status_t mg_level_n(mg_handle h, int level, int *n) {
    if (!h || !n) return fail(MG_ERR_ARG, "null argument");
    if (h->batched) return fail(MG_ERR_STATE, "not available on a batched handle");
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
    if (h->batched || h->nrhs) return fail(MG_ERR_STATE, "not available on a batched or many-right-hand-side handle");
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
    if (h->batched || h->nrhs) return fail(MG_ERR_STATE, "not available on a batched or many-right-hand-side handle");
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
    if (h->batched || h->nrhs) return fail(MG_ERR_STATE, "not available on a batched or many-right-hand-side handle");
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
        e = level_sweep(h, level, L.prec, bbuf(h, level), cbuf(h, level, cur), cbuf(h, level, cur ^ 1), st);
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
    if (h->batched || h->nrhs) return fail(MG_ERR_STATE, "not available on a batched or many-right-hand-side handle");
    if (!b || !c) return fail(MG_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    LevelPlan &L = h->lv[0];
    HIPCHK(launch_pack(h->dim, L.prec, L.prec, L.n, L.P, b, bbuf(h, 0), st));
    HIPCHK(enq_vcycle(h, st, RHS_B));
    HIPCHK(launch_unpack(h->dim, L.prec, L.prec, L.n, L.P, cbuf(h, 0, h->cur[0]), c, st));
    return MG_OK;
}

}  // extern "C"

// ---- the V-cycle on a library-owned scratch array (mg_noalloc.hip) ----------
namespace mg {

mg_status_t set_error(mg_status_t s, const char *msg) { return fail(s, "%s", msg); }

mg_status_t vcycle_scratch_need(mg_handle h, size_t *bytes) {
    if (!h || !bytes) return fail(MG_ERR_ARG, "null argument");
    if (h->batched || h->nrhs) return fail(MG_ERR_STATE, "not available on a batched or many-right-hand-side handle");
    *bytes = h->vc_bytes;
    return MG_OK;
}

mg_status_t vcycle_in(mg_handle h, void *ws, size_t cap, const void *b, void *c, void *stream) {
    size_t need = 0;
    mg_status_t s = vcycle_scratch_need(h, &need);
    if (s != MG_OK) return s;
    if (!ws || !b || !c) return fail(MG_ERR_ARG, "null argument");
    if (need > cap) return fail(MG_ERR_WORKSPACE, "a V-cycle of this handle needs %zu bytes, more than %zu", need, cap);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the handle's own workspace and level roles stay as they were
    char *keep_ws = h->ws;
    int keep_cur[32];
    std::memcpy(keep_cur, h->cur, sizeof keep_cur);
    h->ws = static_cast<char *>(ws);
    const LevelPlan &L = h->lv[0];
    // ghost cells must read zero, and the array keeps the last call's values
    hipError_t e = launch_fill_zero(ws, align_up(need, 16), st);
    if (e == hipSuccess) e = launch_pack(h->dim, L.prec, L.prec, L.n, L.P, b, bbuf(h, 0), st);
    if (e == hipSuccess) e = enq_vcycle(h, st, RHS_B);
    if (e == hipSuccess) e = launch_unpack(h->dim, L.prec, L.prec, L.n, L.P, cbuf(h, 0, h->cur[0]), c, st);
    h->ws = keep_ws;
    std::memcpy(h->cur, keep_cur, sizeof keep_cur);
    if (e != hipSuccess) return fail(MG_ERR_HIP, "V-cycle launch failed: %s", hipGetErrorString(e));
    return MG_OK;
}

}  // namespace mg

extern "C" {

mg_status_t ir_solve(mg_handle h, const double *b, double *u, mg_stats_t *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (h->batched) return fail(MG_ERR_STATE, "use ir_solve_batched on a batched handle");
    if (h->nrhs) return fail(MG_ERR_STATE, "use ir_solve_multi on a many-right-hand-side handle");
    if (!b || !u) return fail(MG_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    LevelPlan &L = h->lv[0];
    const double hh = 1.0 / (double)(L.n + 1);
    const double inv_h2 = 1.0 / (hh * hh);
    const int D = h->dim;
    const int scaling = h->ascale;
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
    h->rpar = 0;
    h->pending = 0;
    h->u_zero = false;
    if (h->defer) HIPCHK(launch_fill_zero(h->ws + h->off_dctr, 16, st));
    if (h->opt.use_initial_guess) {
        HIPCHK(finest_resid(h, b, nullptr, nullptr, nullptr, st));
    } else {
        HIPCHK(finest_resid(h, b, nullptr, Rbuf(h), nullptr, st));
        // with postponed updates nothing reads u before the first flush,
        // which then starts from zero (enq_flush)
        if (h->defer) h->u_zero = true;
        else HIPCHK(launch_fill_zero(Ubuf(h), align_up(L.elems * sizeof(double), 16), st));
    }
    const int fparts = flat_blocks(points(D, L.n));
    HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
    HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double nb = h->host_scal[2];
    if (!std::isfinite(nb) || nb == 0.0) HIPCHK(enq_flush(h, st));  // u = 0 in the handle too
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
        HIPCHK(finest_resid(h, b, Ubuf(h), Rbuf(h), nullptr, st));
        HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
        HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    const bool graph = h->opt.use_graph && !h->prof;
    if (graph) {
        s = ensure_graph(h);
        if (s != MG_OK) return s;
    }
    if (!h->ev_norm) HIPCHK(hipEventCreateWithFlags(&h->ev_norm, hipEventDisableTiming));
    int k = 0;
    bool recursive = false;      // whether R holds a recursively updated residual
    bool cycle_queued = false;   // the V-cycle of the next step is already on the stream
    double prev_rn = -1.0;
    mg_status_t result = MG_OK;
    double rel = h->host_scal[2] / nb;
    auto launch = [&](bool cycle) -> hipError_t {
        if (graph) {
            if (h->rpar) return hipGraphLaunch(cycle ? h->gexec_p1 : h->gexec2_p1, st);
            return hipGraphLaunch(cycle ? h->gexec : h->gexec2, st);
        }
        return cycle ? enq_cycle(h, st) : enq_update(h, st);
    };
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
            // confirm with the residual recomputed from u (a queued V-cycle
            // only wrote level vectors and is discarded)
            cycle_queued = false;
            HIPCHK(enq_flush(h, st));
            HIPCHK(finest_resid(h, b, Ubuf(h), Rbuf(h), u, st));
            HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
            HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            recursive = false;
            prev_rn = -1.0;
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
        hipError_t e = hipSuccess;
        if (!cycle_queued) e = launch(true);
        if (e == hipSuccess) e = launch(false);
        if (e == hipSuccess) e = hipEventRecord(h->ev_norm, st);
        if (e == hipSuccess) e = after_update(h, st);
        // Queue the next step's V-cycle before reading this step's norm when
        // the residual is unlikely to reach the tolerance in this step (the
        // prediction uses the last contraction factor; a wrong guess costs
        // one discarded V-cycle, never a different result).
        cycle_queued = false;
        if (e == hipSuccess && k + 1 < h->opt.max_iter) {
            const double rho = prev_rn > 0.0 ? std::min(1.0, rn / prev_rn) : 0.5;
            if (rn * rho > 8.0 * h->opt.rtol * nb) {
                e = launch(true);
                cycle_queued = e == hipSuccess;
            }
        }
        if (e != hipSuccess) return fail(MG_ERR_HIP, "refinement step launch failed: %s", hipGetErrorString(e));
        HIPCHK(hipEventSynchronize(h->ev_norm));
        prev_rn = rn;
        recursive = true;
        ++k;
    }
    if (cycle_queued) HIPCHK(hipStreamSynchronize(st));
    // final: recompute the true residual and copy u out
    HIPCHK(enq_flush(h, st));
    HIPCHK(finest_resid(h, b, Ubuf(h), Rbuf(h), u, st));
    HIPCHK(launch_finalize(part(h), fparts, scal(h), scaling, st));
    HIPCHK(hipMemcpyAsync(h->host_scal, scal(h), 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rel = h->host_scal[2] / nb;
    finish_stats(k, rel);
    return result;
}

mg_status_t mg_set_shape(mg_handle h, int level, int kind, const int *p, int np) {
    if (!h || !p) return fail(MG_ERR_ARG, "null argument");
    if (h->batched || h->nrhs) return fail(MG_ERR_STATE, "not available on a batched or many-right-hand-side handle");
    if (h->q1) {
        // the LDS-staged kernels' {ty, zc}: the sweep (MG_SHAPE_SWEEP), the
        // residual (MG_SHAPE_RESTRICT), the update (MG_SHAPE_UPDATE, level 0)
        const int k = q1_kind(kind);
        if (k < 0) return fail(MG_ERR_STATE, "a Q1 handle has sweep, residual and update shapes only");
        if (level < 0 || level >= h->nl - 1 || (k == 2 && level != 0))
            return fail(MG_ERR_ARG, "level %d has no such Q1 kernel", level);
        if (np != 2 && !(np == 3 && k == 1))
            return fail(MG_ERR_ARG, "a Q1 shape is {ty, zc} ({0, 0}: the built-in one), the residual's {ty, zc[, split]}");
        LevelPlan &L = h->lv[level];
        const Q1Shape q{p[0], p[1], np == 3 ? p[2] : 0};
        if (!q1_shape_ok(h->dim, L.prec, L.n, L.P, k, q))
            return fail(MG_ERR_ARG,
                        "Q1 shape {%d, %d, split %d} not valid on level %d (3-D levels in a 2-byte format only; the "
                        "fused residual + restriction takes even ty and zc)",
                        q.ty, q.zc, q.split, level);
        L.q1s[k] = q;
        set_fused(h, h->fused);  // the update's partial count
        drop_graph(h);
        return MG_OK;
    }
    if (kind == MG_SHAPE_TAIL) {
        if (np != 1 || (p[0] != 0 && p[0] != 1)) return fail(MG_ERR_ARG, "the tail shape is {0|1}");
        h->tail_on = p[0] != 0;
        drop_graph(h);
        return MG_OK;
    }
    if (kind == MG_SHAPE_FUSE_SR) {
        if (level < 0 || level >= h->nl - 1) return fail(MG_ERR_ARG, "level %d has no restriction", level);
        if ((np != 1 && np != 3 && np != 4) || (p[0] != 0 && p[0] != 1) || (np == 4 && p[3] != 0 && p[3] != 1))
            return fail(MG_ERR_ARG, "the fused smoothing + restriction shape is {on (0|1)[, tyc, zcc[, lds16 (0|1)]]}");
        if (np >= 3) {
            const RShape r{8, p[1], p[2], np == 4 && p[3] ? 4 : 3};
            if (!smooth_restrict_ok(h->lv[level].P, h->lv[level].prec, r))
                return fail(MG_ERR_ARG, "fused smoothing + restriction shape {tyc, zcc} not valid here");
            (level == 0 ? h->srsh : h->lv[level].fsrsh) = r;
        }
        if (level == 0) {
            h->fuse_sr_on = p[0] != 0;
            set_fused_sr(h, h->fuse_sr_on);
        } else {
            h->lv[level].fsr_on = p[0] != 0;
            set_fused_srb(h, level, h->lv[level].fsr_on);
        }
        drop_graph(h);
        return MG_OK;
    }
    if (kind == MG_SHAPE_FUSE) {
        if ((np != 1 && np != 5 && np != 6) || (p[0] != 0 && p[0] != 1))
            return fail(MG_ERR_ARG, "the fused-update shape is {on (0|1)[, V, zc, xcd, ty[, from_r]]}");
        if (np >= 5) {
            const Shape f{p[1], p[2], 256, p[3], p[4]};
            if (h->nl < 2 || !sweep_update_ok(h->lv[0].P, h->lv[0].prec, f) || (f.xcd != 0 && f.xcd != 1))
                return fail(MG_ERR_ARG, "fused-update shape {V=4, zc, xcd, ty} not valid here");
            if (np == 6 && (p[5] < 0 || p[5] > 1 || (p[5] == 0 && finest_alias(h)) || (p[5] == 1 && !h->off_R2)))
                return fail(MG_ERR_ARG, "from_r = %d not valid here (0: read b, 1: form b from r)", p[5]);
            h->fsh = f;
            if (np == 6) h->su_r = p[5] != 0;
        }
        h->fuse_on = p[0] != 0;
        set_fused(h, h->fuse_on);
        drop_graph(h);
        return MG_OK;
    }
    if (level < 0 || level >= h->nl - 1) return fail(MG_ERR_ARG, "level %d has no launch shape", level);
    LevelPlan &L = h->lv[level];
    const int D = h->dim;
    const bool stencil_kind = kind == MG_SHAPE_STENCIL || kind == MG_SHAPE_UPDATE || kind == MG_SHAPE_SMOOTH ||
                              kind == MG_SHAPE_SWEEP || kind == MG_SHAPE_PROLONG;
    if (stencil_kind) {
        if (kind == MG_SHAPE_UPDATE && level != 0) return fail(MG_ERR_ARG, "the update shape exists on level 0 only");
        if (np < 5 || np > 7)
            return fail(MG_ERR_ARG, "stencil shape takes 5 to 7 values {V, zc, bs, xcd, ty[, dp[, sg]]}");
        Shape s{p[0], p[1], p[2], p[3], p[4], np >= 6 ? p[5] : 1, np == 7 ? p[6] : 1};
        if (s.dp < 1 || s.dp > 2 || (s.dp == 2 && s.ty == 0))
            return fail(MG_ERR_ARG, "dp must be 1, or 2 with ty > 0");
        if (s.sg != 0 && s.sg != 1) return fail(MG_ERR_ARG, "sg must be 0 or 1");
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
            set_fused(h, h->fused);
        } else if (kind == MG_SHAPE_STENCIL) {
            L.shs[SH_SMOOTH] = L.shs[SH_SWEEP] = L.shs[SH_PROLONG] = s;
        } else {
            L.shs[kind == MG_SHAPE_SMOOTH ? SH_SMOOTH : kind == MG_SHAPE_SWEEP ? SH_SWEEP : SH_PROLONG] = s;
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
    if (h->batched) return fail(MG_ERR_STATE, "a batched handle's shapes are read with mg_get_instance_shape");
    if (h->nrhs) {
        if (level < 0 || level >= h->nl - 1) return fail(MG_ERR_ARG, "level %d has no launch shape", level);
        return level_shape(h->lv[level], level, kind, p, np);
    }
    if (kind == MG_SHAPE_TAIL) {
        if (np < 1) return fail(MG_ERR_ARG, "too few values");
        p[0] = h->tail_on ? 1 : 0;
        return MG_OK;
    }
    if (h->q1) {
        // the {ty, zc} the LDS-staged kernel uses ({0, 0}: the level has none)
        const int k = q1_kind(kind);
        if (k < 0) return fail(MG_ERR_STATE, "a Q1 handle has sweep, residual and update shapes only");
        if (level < 0 || level >= h->nl - 1 || (k == 2 && level != 0))
            return fail(MG_ERR_ARG, "level %d has no such Q1 kernel", level);
        if (np < 2) return fail(MG_ERR_ARG, "too few values");
        const LevelPlan &L = h->lv[level];
        const Q1Shape u = q1_shape_used(h->dim, L.prec, L.n, L.P, k, L.q1s[k]);
        p[0] = u.ty, p[1] = u.zc;
        if (np >= 3) p[2] = k == 1 ? u.split : 0;
        return MG_OK;
    }
    if (kind == MG_SHAPE_FUSE_SR) {
        if (level < 0 || level >= h->nl - 1) return fail(MG_ERR_ARG, "level %d has no restriction", level);
        if (np < 1) return fail(MG_ERR_ARG, "too few values");
        const RShape &r = level == 0 ? h->srsh : h->lv[level].fsrsh;
        p[0] = (level == 0 ? h->fused_sr : h->lv[level].fsr) ? 1 : 0;
        if (np >= 3) p[1] = r.tyc, p[2] = r.zcc;
        if (np >= 4) p[3] = r.pipe == 4 ? 1 : 0;
        return MG_OK;
    }
    if (kind == MG_SHAPE_FUSE) {
        if (np < 1) return fail(MG_ERR_ARG, "too few values");
        p[0] = h->fused ? 1 : 0;
        if (np >= 5) p[1] = h->fsh.V, p[2] = h->fsh.zc, p[3] = h->fsh.xcd, p[4] = h->fsh.ty;
        if (np >= 6) p[5] = h->su_r ? 1 : 0;
        return MG_OK;
    }
    if (level < 0 || level >= h->nl - 1) return fail(MG_ERR_ARG, "level %d has no launch shape", level);
    return level_shape(h->lv[level], level, kind, p, np);
}

mg_status_t mg_get_instance_shape(mg_handle h, int inst, int level, int kind, int *p, int np) {
    if (!h || !p) return fail(MG_ERR_ARG, "null argument");
    if (!h->batched) return fail(MG_ERR_STATE, "not a batched handle");
    if (inst < 0 || inst >= (int)h->inst.size()) return fail(MG_ERR_ARG, "no instance %d", inst);
    const auto &I = h->inst[inst];
    if (level < 0 || level >= I.nl - 1) return fail(MG_ERR_ARG, "level %d has no launch shape", level);
    if (kind == MG_SHAPE_UPDATE) {
        if (level != 0) return fail(MG_ERR_ARG, "the update runs on level 0 only");
        LevelPlan L = I.lv[0];
        L.osh = I.osh;
        return level_shape(L, 0, kind, p, np);
    }
    return level_shape(I.lv[level], level, kind, p, np);
}

mg_status_t mg_bandwidth_probe(void *dst, const void *src, size_t bytes, int kind, int blocks, void *stream) {
    if (!dst || !src || kind < 0 || kind > 7 || blocks < 1) return fail(MG_ERR_ARG, "bad argument");
    const bool mix = kind == 3 || kind == 6 || kind == 7;
    if (bytes % (mix ? 32 : 16)) return fail(MG_ERR_ARG, "bytes must be a multiple of 16 (32 for the update mix)");
    HIPCHK(launch_probe(dst, src, bytes, kind, blocks, static_cast<unsigned *>(dst), static_cast<hipStream_t>(stream)));
    return MG_OK;
}

mg_status_t mg_profile_step(mg_handle h, void *stream, int cap, int *count, const char **names, double *ms,
                            double *bytes, int *levels_out) {
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!count || cap < 0) return fail(MG_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (h->batched) {
        // profile a step of every instance from its current state
        const int ni = (int)h->inst.size();
        for (int i = 0; i < ni; ++i) h->host_active[i] = 1;
        HIPCHK(hipMemcpyAsync(h->ws + h->off_active, h->host_active, sizeof(int) * ni, hipMemcpyHostToDevice, st));
    }
    h->prof = true;
    h->recs.clear();
    if (h->nrhs) {
        for (int k = 0; k < h->nrhs; ++k) h->host_mask[k] = 1;
        HIPCHK(hipMemcpyAsync(h->ws + h->off_act, h->host_mask, sizeof(int) * h->nrhs, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    hipError_t e = h->batched ? enq_batched_step(h, st) : h->nrhs ? enq_multi_step(h, st) : enq_step(h, st);
    if (e == hipSuccess && !h->batched && !h->nrhs) {
        // a postponed update is added to u at once, so that the step leaves
        // the state a real one would after its flush (timed as defer_flush)
        e = after_update(h, st);
        if (e == hipSuccess) e = enq_flush(h, st);
    }
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

// ============================================================================
// Batched instances
// ============================================================================
namespace {

// Batched launch shapes: the LDS-plane kernels wherever the single-grid
// default uses them (pitch >= 16), else the register-queue kernel with a
// fixed block size of 256.
// `copies`: instances of this size in the batch, which share each launch.
// Longer z marches amortise a tile's pipeline prologue; the plane chunk is
// chosen so that a launch still has about 4096 tiles.
Shape batched_shape(int P, int prec, int copies) {
    Shape s = pick_shape(3, P, prec);
    if (s.ty > 0) {
        const long ytiles = (P - 1 + s.ty - 1) / s.ty;
        const long nch = std::max(1L, (4096 + ytiles * copies - 1) / (ytiles * copies));
        s.zc = std::max(1, std::min(32, (int)((P - 1 + nch - 1) / nch)));
        return s;
    }
    s.V = (P >= 8 && prec != P_F64) ? 8 : 4;
    s.bs = 256;
    const long per_chunk = (long)(P / s.V) * P;
    const long nch = ((1L << 17) + per_chunk - 1) / per_chunk;
    s.zc = std::max(1, std::min((int)((P - 1 + nch - 1) / nch), 32));
    return s;
}

RShape batched_rshape(int P, int pf, int copies) {
    if (P >= 16) {
        RShape r = pick_rshape(3, P, pf);
        if (r.pipe >= 1) {
            const long ytiles = (P / 2 - 1 + r.tyc - 1) / r.tyc;
            const long nzc = std::max(1L, (4096 + ytiles * copies - 1) / (ytiles * copies));
            r.zcc = std::max(1, std::min(16, (int)((P / 2 - 1 + nzc - 1) / nzc)));
            return r;
        }
    }
    RShape r;
    r.V = (P >= 8 && pf != P_F64) ? 8 : 4;
    r.pipe = 0;
    const int TXR = P / r.V, Pc = P / 2;
    const size_t acc = pf == P_F64 ? 8 : 4;
    int tyc = std::max(1, std::min(7, Pc - 1));
    while (tyc > 1 && ((2 * tyc + 1) * TXR > 1024 || 2 * (size_t)(2 * tyc + 1) * P * acc > 65536)) --tyc;
    r.tyc = tyc;
    const int ytiles = (Pc - 1 + tyc - 1) / tyc;
    const int nzc = std::max(1, (256 + ytiles - 1) / ytiles);
    r.zcc = std::max(1, (Pc - 1 + nzc - 1) / nzc);
    return r;
}

// Work items of one instance's stencil launch with shape s.
int batched_stencil_blocks(int P, const Shape &s) {
    if (s.ty > 0) return ((P - 1 + s.ty - 1) / s.ty) * ((P - 1 + s.zc - 1) / s.zc);
    return stencil_blocks(3, P, s);
}

int bprec_of(const mg_ctx *h, int i, int l) {
    return l == h->inst[i].nl - 1 ? h->bprec[h->Lmax - 1] : h->bprec[l];
}

// Build the batched stage list and the descriptor / item image for the
// workspace at `base` (nullptr only to size the image).
void build_batched_plan(mg_ctx *h, char *base) {
    const int ni = (int)h->inst.size();
    const bool alias = h->bprec[0] == P_F64 && !h->opt.residual_scaling;
    std::vector<BDesc> descs;
    std::vector<BItem> items;
    std::vector<BFin> fins;
    h->bl.clear();
    std::vector<std::vector<int>> cur(ni, std::vector<int>(h->Lmax, 0));
    // addresses are formed as integers so that sizing with base == nullptr is defined
    auto at = [&](size_t off) { return reinterpret_cast<char *>(reinterpret_cast<uintptr_t>(base) + off); };
    auto B = [&](int i, int l) -> void * { return at(h->inst[i].lv[l].off_b); };
    auto C = [&](int i, int l, int w) -> void * { return at(h->inst[i].lv[l].off_c[w]); };
    auto Rp = [&](int i) { return reinterpret_cast<double *>(at(h->inst[i].off_R)); };
    auto Up = [&](int i) { return reinterpret_cast<double *>(at(h->inst[i].off_U)); };
    auto Sp = [&](int i) { return reinterpret_cast<double *>(at(h->off_scal_all + 32 * (size_t)i)); };
    auto rhs = [&](int i, int l) -> const void * { return (l == 0 && alias) ? (const void *)Rp(i) : B(i, l); };
    // Launches group descriptors of one kernel form: register-queue stencil
    // (what 0), register restriction (1), LDS-plane stencil (4, one pitch
    // per launch) and pipelined restriction (5, one pitch per launch).
    struct Pend {
        BDesc d;
        int what, V, pc, nblk, threads;
        size_t lds;
        bool xsh;
    };
    auto flush = [&](int kind, int pf, const char *name, int level, std::vector<Pend> &pend,
                     double bytes_per_point) {
        // the LDS forms need one block size per launch: same pitch and rows
        struct Key {
            int what, V, pc, P, rows;
            bool xsh;
            bool operator==(const Key &o) const {
                return what == o.what && V == o.V && pc == o.pc && P == o.P && rows == o.rows && xsh == o.xsh;
            }
        };
        auto key_of = [](const Pend &p) {
            if (p.what == 4) return Key{p.what, p.V, p.pc, p.d.P, p.d.ty, false};
            if (p.what == 5) return Key{p.what, p.V, p.pc, p.d.P, p.d.tyc, p.xsh};
            return Key{p.what, p.V, p.pc, 0, 0, false};
        };
        std::vector<Key> keys;
        for (auto &p : pend)
            if (std::find(keys.begin(), keys.end(), key_of(p)) == keys.end()) keys.push_back(key_of(p));
        for (auto &k : keys) {
            mg_ctx::BLaunch L{};
            L.what = k.what, L.kind = k.what == 5 ? (k.xsh ? 1 : 0) : kind, L.V = k.V, L.pf = pf, L.pc = k.pc;
            L.off_desc = descs.size(), L.off_items = items.size();
            L.name = name, L.level = level;
            int maxthreads = 0;
            size_t maxlds = 0;
            double pts = 0;
            for (auto &p : pend) {
                if (!(key_of(p) == k)) continue;
                const int di = (int)(descs.size() - L.off_desc);
                descs.push_back(p.d);
                for (int b = 0; b < p.nblk; ++b) items.push_back(BItem{di, b});
                pts += (double)(p.d.P - 1) * (p.d.P - 1) * (p.d.P - 1);
                maxthreads = std::max(maxthreads, p.threads);
                maxlds = std::max(maxlds, p.lds);
            }
            L.ndesc = (int)(descs.size() - L.off_desc);
            L.nitems = (int)(items.size() - L.off_items);
            L.grid = std::max(1, std::min(L.nitems, k.what == 0 ? 4096 : 2048));
            // the register restriction tolerates extra threads; the LDS forms
            // take exactly their row groups
            L.threads = k.what == 0 ? 256 : k.what == 1 ? ((maxthreads + 63) / 64) * 64 : maxthreads;
            L.lds = maxlds;
            L.bytes = pts * bytes_per_point;
            h->bl.push_back(L);
        }
        pend.clear();
    };
    // a stencil-stage descriptor with the form that shape sh selects
    auto stencil_pend = [&](BDesc x, const Shape &sh, int P, int prec, int pc) {
        x.P = P, x.zc = sh.zc, x.nchunks = (P - 1 + sh.zc - 1) / sh.zc;
        Pend p{};
        p.V = sh.V, p.pc = pc;
        if (sh.ty > 0) {
            x.ty = sh.ty, x.ytiles = (P - 1 + sh.ty - 1) / sh.ty;
            p.what = 4;
            p.threads = (sh.ty + 2) * (P / sh.V);
            p.lds = march_lds_bytes(P, sh.ty, prec_bytes(prec));
        } else {
            p.what = 0;
            p.threads = 256;
        }
        p.nblk = batched_stencil_blocks(P, sh);
        p.d = x;
        return p;
    };
    auto restrict_pend = [&](BDesc x, const RShape &r, int P, int pf, int pc) {
        x.P = P, x.tyc = r.tyc, x.zcc = r.zcc, x.ytiles = (P / 2 - 1 + r.tyc - 1) / r.tyc;
        Pend p{};
        p.V = r.V, p.pc = pc, p.xsh = r.pipe >= 2;
        p.nblk = restrict_blocks(3, P, r);
        if (r.pipe >= 1) {
            const RShape rr{r.V, r.tyc, r.zcc, p.xsh ? 3 : 1};
            p.what = 5;
            p.threads = (2 * r.tyc + 3) * (P / r.V);
            p.lds = restrict_lds_bytes(3, P, pf, rr);
        } else {
            p.what = 1;
            p.threads = (2 * r.tyc + 1) * (P / r.V);
            p.lds = 2 * (size_t)(2 * r.tyc + 1) * P * (pf == P_F64 ? 8 : 4);
        }
        p.d = x;
        return p;
    };
    std::vector<Pend> pend;
    for (int d = 0; d + 1 < h->Lmax; ++d) {
        const int pf = h->bprec[d];
        const double s = (double)prec_bytes(pf);
        // first pre-smoothing (two sweeps fused)
        for (int i = 0; i < ni; ++i) {
            if (d > h->inst[i].nl - 2) continue;
            const LevelPlan &L = h->inst[i].lv[d];
            BDesc x{};
            x.b = (d == 0) ? (const void *)Rp(i) : B(i, d);
            x.cout = C(i, d, 0);
            x.bout = B(i, d);
            x.scal = Sp(i);
            x.inst = i;
            pend.push_back(stencil_pend(x, L.shs[SH_SMOOTH], L.P, pf, P_F64));
            cur[i][d] = 0;
        }
        const bool scaled = d == 0 && !alias;
        flush(scaled ? BK_SMOOTH2_SCALED : BK_SMOOTH2, pf, scaled ? "smooth2_scaled" : "smooth2", d, pend,
              scaled ? 8 + 2 * s : 2 * s);
        for (int k = 2; k < h->opt.nu1; ++k) {
            for (int i = 0; i < ni; ++i) {
                if (d > h->inst[i].nl - 2) continue;
                const LevelPlan &L = h->inst[i].lv[d];
                BDesc x{};
                x.b = rhs(i, d), x.cin = C(i, d, cur[i][d]), x.cout = C(i, d, cur[i][d] ^ 1), x.inst = i;
                pend.push_back(stencil_pend(x, L.shs[SH_SWEEP], L.P, pf, P_F64));
                cur[i][d] ^= 1;
            }
            flush(BK_SWEEP, pf, "sweep", d, pend, 3 * s);
        }
        for (int i = 0; i < ni; ++i) {
            if (d > h->inst[i].nl - 2) continue;
            const LevelPlan &L = h->inst[i].lv[d];
            BDesc x{};
            x.b = rhs(i, d), x.cin = C(i, d, cur[i][d]), x.cout = B(i, d + 1), x.inst = i;
            pend.push_back(restrict_pend(x, L.rsh, L.P, pf, bprec_of(h, i, d + 1)));
        }
        flush(0, pf, "resid_restrict", d, pend, 2 * s);
    }
    for (int i = 0; i < ni; ++i) {
        const int lb = h->inst[i].nl - 1;
        BDesc x{};
        x.b = B(i, lb), x.cout = C(i, lb, 0), x.inst = i;
        cur[i][lb] = 0;
        descs.push_back(x);
    }
    {
        mg_ctx::BLaunch L{};
        L.what = 2, L.pf = h->bprec[h->Lmax - 1], L.off_desc = descs.size() - ni, L.ndesc = ni, L.name = "coarse_solve";
        L.level = h->Lmax - 1;
        h->bl.push_back(L);
    }
    for (int d = h->Lmax - 2; d >= 0; --d) {
        const int pf = h->bprec[d];
        const double s = (double)prec_bytes(pf);
        for (int i = 0; i < ni; ++i) {
            if (d > h->inst[i].nl - 2) continue;
            const LevelPlan &L = h->inst[i].lv[d];
            BDesc x{};
            x.b = rhs(i, d), x.cin = C(i, d, cur[i][d]), x.ec = C(i, d + 1, cur[i][d + 1]);
            x.cout = C(i, d, cur[i][d] ^ 1), x.inst = i;
            pend.push_back(stencil_pend(x, L.shs[SH_PROLONG], L.P, pf, bprec_of(h, i, d + 1)));
            cur[i][d] ^= 1;
        }
        flush(BK_PROLONG, pf, "prolong_sweep", d, pend, 3 * s);
        for (int k = 1; k < h->opt.nu2; ++k) {
            for (int i = 0; i < ni; ++i) {
                if (d > h->inst[i].nl - 2) continue;
                const LevelPlan &L = h->inst[i].lv[d];
                BDesc x{};
                x.b = rhs(i, d), x.cin = C(i, d, cur[i][d]), x.cout = C(i, d, cur[i][d] ^ 1), x.inst = i;
                pend.push_back(stencil_pend(x, L.shs[SH_SWEEP], L.P, pf, P_F64));
                cur[i][d] ^= 1;
            }
            flush(BK_SWEEP, pf, "sweep", d, pend, 3 * s);
        }
    }
    double *part_base = reinterpret_cast<double *>(at(h->off_part));
    for (int i = 0; i < ni; ++i) {
        const LevelPlan &L = h->inst[i].lv[0];
        const double hh = 1.0 / (double)(L.n + 1);
        BDesc x{};
        x.cin = C(i, 0, cur[i][0]), x.R = Rp(i), x.U = Up(i), x.scal = Sp(i), x.h2 = hh * hh;
        x.part_off = h->inst[i].part_off, x.inst = i;
        pend.push_back(stencil_pend(x, h->inst[i].osh, L.P, h->bprec[0], P_F64));
        fins.push_back(
            BFin{part_base + 2 * (size_t)h->inst[i].part_off, batched_stencil_blocks(L.P, h->inst[i].osh), Sp(i),
                 h->inst[i].ascale});
    }
    flush(BK_OUTER, h->bprec[0], "ir_update", 0, pend, 32 + (double)prec_bytes(h->bprec[0]));
    {
        mg_ctx::BLaunch L{};
        L.what = 3, L.name = "norm_finalize", L.level = 0;
        h->bl.push_back(L);
    }
    // image: descriptors, then items, then finalize records
    const size_t nd = descs.size() * sizeof(BDesc), nit = items.size() * sizeof(BItem), nf = fins.size() * sizeof(BFin);
    const size_t off_items = align_up(nd, 256), off_fin = off_items + align_up(nit, 256);
    h->bmeta_bytes = off_fin + align_up(nf, 256);
    if (base) {
        std::vector<unsigned char> img(h->bmeta_bytes, 0);
        std::memcpy(img.data(), descs.data(), nd);
        std::memcpy(img.data() + off_items, items.data(), nit);
        std::memcpy(img.data() + off_fin, fins.data(), nf);
        const BDesc *dd = reinterpret_cast<const BDesc *>(at(h->off_bmeta));
        const BItem *ii = reinterpret_cast<const BItem *>(at(h->off_bmeta + off_items));
        for (auto &L : h->bl) {
            L.off_desc = reinterpret_cast<size_t>(dd + L.off_desc);
            L.off_items = reinterpret_cast<size_t>(ii + L.off_items);
        }
        h->off_fin = h->off_bmeta + off_fin;
        // the caller copies img into the workspace
        h->bmeta_img_tmp = std::move(img);
    }
}

hipError_t enq_batched_step(mg_ctx *h, hipStream_t st) {
    const int *act = reinterpret_cast<const int *>(h->ws + h->off_active);
    double *part_base = reinterpret_cast<double *>(h->ws + h->off_part);
    for (auto &L : h->bl) {
        const BDesc *d = reinterpret_cast<const BDesc *>(L.off_desc);
        const BItem *it = reinterpret_cast<const BItem *>(L.off_items);
        if (L.what == 0) {
            RUN(h, st, L.name, L.level, L.bytes,
                launch_batched_stencil(L.kind, L.V, L.pf, L.pc, d, it, L.nitems, act, h->opt.omega, part_base,
                                       L.grid, st));
        } else if (L.what == 4) {
            RUN(h, st, L.name, L.level, L.bytes,
                launch_batched_march(L.kind, L.V, L.pf, L.pc, d, it, L.nitems, act, h->opt.omega, part_base, L.grid,
                                     L.threads, L.lds, st));
        } else if (L.what == 5) {
            RUN(h, st, L.name, L.level, L.bytes,
                launch_batched_restrict2(L.V, L.pf, L.pc, L.kind == 1, d, it, L.nitems, act, L.grid, L.threads, L.lds,
                                         st));
        } else if (L.what == 1) {
            RUN(h, st, L.name, L.level, L.bytes,
                launch_batched_restrict(L.V, L.pf, L.pc, d, it, L.nitems, act, L.grid, L.threads, L.lds, st));
        } else if (L.what == 2) {
            RUN(h, st, L.name, L.level, 0.0, launch_batched_coarse(L.pf, d, L.ndesc, act, st));
        } else {
            RUN(h, st, L.name, 0, 0.0,
                launch_batched_finalize(reinterpret_cast<const BFin *>(h->ws + h->off_fin), (int)h->inst.size(), act,
                                        st));
        }
    }
    return hipMemcpyAsync(h->host_scal_all, h->ws + h->off_scal_all, 4 * sizeof(double) * h->inst.size(),
                          hipMemcpyDeviceToHost, st);
}

// ---- batched autotuner ---------------------------------------------------------
// Launch shapes are chosen per class of levels (pitch and format): every level
// of the class, in every instance, takes the class's shape, and the choice
// only changes how the work is cut (every shape forms the same roundings).  A
// candidate is timed as a whole batched refinement step with every instance
// active, class by class from the largest pitch, stencil shape first, then the
// restriction shape.
struct BClass {
    int P, prec;
};

std::vector<BClass> batched_classes(const mg_ctx *h) {
    std::vector<BClass> cl;
    for (const auto &I : h->inst)
        for (int l = 0; l + 1 < I.nl; ++l) {
            const LevelPlan &L = I.lv[l];
            if (L.P < 16) continue;
            bool seen = false;
            for (const auto &c : cl) seen = seen || (c.P == L.P && c.prec == L.prec);
            if (!seen) cl.push_back(BClass{L.P, L.prec});
        }
    std::sort(cl.begin(), cl.end(), [](const BClass &a, const BClass &b) { return a.P > b.P || (a.P == b.P && a.prec < b.prec); });
    return cl;
}

template <class F> void for_class(mg_ctx *h, const BClass &c, F &&f) {
    for (auto &I : h->inst)
        for (int l = 0; l + 1 < I.nl; ++l)
            if (I.lv[l].P == c.P && I.lv[l].prec == c.prec) f(I.lv[l]);
}

std::string batched_tune_key(const mg_ctx *h) {
    const std::string dk = device_key();
    if (dk.empty()) return dk;
    std::string k = dk + "|batched|nu" + std::to_string(h->opt.nu1) + "," + std::to_string(h->opt.nu2) + "|sc" +
                    std::to_string(h->opt.residual_scaling) + "|p";
    for (int p : h->bprec) k += std::to_string(p);
    std::vector<int> ns;
    for (const auto &I : h->inst) ns.push_back(I.n);
    std::sort(ns.begin(), ns.end());
    for (size_t i = 0; i < ns.size();) {
        size_t j = i;
        while (j < ns.size() && ns[j] == ns[i]) ++j;
        k += "|" + std::to_string(ns[i]) + "x" + std::to_string(j - i);
        i = j;
    }
    return k;
}

// Build the plan for the current shapes and copy its descriptors into the
// workspace; MG_ERR_WORKSPACE (nothing copied) when they exceed the room
// reserved for them.
mg_status_t batched_upload(mg_ctx *h) {
    build_batched_plan(h, nullptr);
    if (h->bmeta_bytes > h->bmeta_cap)
        return fail(MG_ERR_WORKSPACE, "batched plan of %zu bytes exceeds its %zu", h->bmeta_bytes, h->bmeta_cap);
    build_batched_plan(h, h->ws);
    HIPCHK(hipMemcpy(h->ws + h->off_bmeta, h->bmeta_img_tmp.data(), h->bmeta_img_tmp.size(), hipMemcpyHostToDevice));
    h->bmeta_img_tmp.clear();
    return MG_OK;
}

// state: per class {P, prec, stencil V, zc, ty, restriction V, tyc, zcc, pipe}
constexpr int kBClassInts = 9;

bool apply_batched_state(mg_ctx *h, const std::vector<int> &v) {
    const std::vector<BClass> cl = batched_classes(h);
    if (v.size() != cl.size() * kBClassInts) return false;
    for (size_t c = 0; c < cl.size(); ++c) {
        const int *q = v.data() + c * kBClassInts;
        if (q[0] != cl[c].P || q[1] != cl[c].prec) return false;
        LevelPlan probe;
        probe.P = cl[c].P, probe.prec = cl[c].prec;
        const Shape sh{q[2], q[3], 256, 1, q[4]};
        const RShape rs{q[5], q[6], q[7], q[8]};
        if (!stencil_ok(h, probe, sh) || !restrict_ok(h, probe, rs)) return false;
    }
    for (size_t c = 0; c < cl.size(); ++c) {
        const int *q = v.data() + c * kBClassInts;
        const Shape sh{q[2], q[3], 256, 1, q[4]};
        const RShape rs{q[5], q[6], q[7], q[8]};
        for_class(h, cl[c], [&](LevelPlan &L) {
            L.shs[SH_SMOOTH] = L.shs[SH_SWEEP] = L.shs[SH_PROLONG] = sh;
            L.rsh = rs;
        });
    }
    return true;
}

mg_status_t autotune_batched(mg_ctx *h, hipStream_t st) {
    const std::string key = batched_tune_key(h);
    std::vector<int> v;
    if (cache_read(key, v) && apply_batched_state(h, v)) return batched_upload(h);
    const int ni = (int)h->inst.size();
    for (int i = 0; i < ni; ++i) h->host_active[i] = 1;
    HIPCHK(hipMemcpy(h->ws + h->off_active, h->host_active, sizeof(int) * ni, hipMemcpyHostToDevice));
    auto step_ms = [&]() -> float {
        if (batched_upload(h) != MG_OK) return 1e30f;
        return time_ms(st, [&]() { return enq_batched_step(h, st); }, 2);
    };
    const std::vector<BClass> cl = batched_classes(h);
    v.clear();
    for (const BClass &c : cl) {
        LevelPlan probe;
        probe.P = c.P, probe.prec = c.prec;
        Shape bs;
        RShape br;
        for_class(h, c, [&](LevelPlan &L) { bs = L.shs[SH_SWEEP], br = L.rsh; });
        float best = step_ms();
        for (int V : {4, 8})
            for (int ty : {0, 2, 4, 6, 10, 14})
                for (int zc : {2, 4, 8, 16, 32}) {
                    const Shape s{V, zc, 256, 1, ty};
                    if ((ty == 0 && zc < 8) || !stencil_ok(h, probe, s)) continue;
                    if (c.prec == P_F64 && V == 8 && ty > 0) continue;  // FP64 rows spill at V = 8
                    for_class(h, c, [&](LevelPlan &L) { L.shs[SH_SMOOTH] = L.shs[SH_SWEEP] = L.shs[SH_PROLONG] = s; });
                    const float t = step_ms();
                    if (t < best) best = t, bs = s;
                }
        for_class(h, c, [&](LevelPlan &L) { L.shs[SH_SMOOTH] = L.shs[SH_SWEEP] = L.shs[SH_PROLONG] = bs; });
        for (int V : {4, 8})
            for (int tyc : {1, 2, 3, 5, 7})
                for (int zcc : {2, 4, 8, 16})
                    for (int pipe : {0, 1, 2}) {
                        const RShape r{V, tyc, zcc, pipe};
                        if (!restrict_ok(h, probe, r)) continue;
                        for_class(h, c, [&](LevelPlan &L) { L.rsh = r; });
                        const float t = step_ms();
                        if (t < best) best = t, br = r;
                    }
        for_class(h, c, [&](LevelPlan &L) { L.rsh = br; });
        v.insert(v.end(), {c.P, c.prec, bs.V, bs.zc, bs.ty, br.V, br.tyc, br.zcc, br.pipe});
    }
    mg_status_t s = batched_upload(h);
    if (s != MG_OK) return s;
    HIPCHK(hipMemsetAsync(h->ws, 0, h->ws_need, st));
    HIPCHK(hipStreamSynchronize(st));
    s = batched_upload(h);  // (the descriptors lie in the workspace just cleared)
    if (s == MG_OK) cache_write(key, v);
    return s;
}

}  // namespace

extern "C" {

mg_status_t mg_setup_batched(mg_handle *out, int dim, int ninst, const int *n, const mg_prec_t *level_prec,
                             const mg_options_t *opt) {
    if (!out || !n) return fail(MG_ERR_ARG, "null argument");
    if (dim != 3) return fail(MG_ERR_SHAPE, "batched instances are 3-D (dim = 3)");
    if (ninst < 1 || ninst > 4096) return fail(MG_ERR_ARG, "ninst must be in 1..4096");
    mg_options_t o;
    mg_default_options(&o);
    if (opt) o = *opt;
    if (o.rescale_half) return fail(MG_ERR_ARG, "rescale_half is only available on single-grid handles");
    if (o.defer_update) return fail(MG_ERR_ARG, "defer_update is only available on single-grid handles");
    if (o.discretization != MG_DISC_FD)
        return fail(MG_ERR_ARG, "the Q1 discretisation is only available on single-grid handles");
    if (o.cycles_per_step != 1)
        return fail(MG_ERR_ARG, "cycles_per_step other than 1 is only available on single-grid handles");
    if (o.nu1 < 2 || o.nu1 > 16 || o.nu2 < 1 || o.nu2 > 16)
        return fail(MG_ERR_ARG, "batched solves need 2 <= nu1 <= 16 and 1 <= nu2 <= 16");
    if (!(o.omega > 0.0 && o.omega < 2.0) || o.max_iter < 0 || !(o.rtol >= 0.0)) return fail(MG_ERR_ARG, "bad options");
    int Lmax = 0;
    for (int i = 0; i < ninst; ++i) {
        if (n[i] < 3 || n[i] > 1023 || ((n[i] + 1) & n[i]) != 0)
            return fail(MG_ERR_SHAPE, "instance %d: n must be 2^m - 1 with 2 <= m <= 10, got %d", i, n[i]);
        int m = 0;
        while ((1 << m) < n[i] + 1) ++m;
        Lmax = std::max(Lmax, m);
    }
    std::vector<int> prec(Lmax, P_F64);
    if (level_prec)
        for (int l = 0; l < Lmax; ++l) {
            if (!valid_prec((int)level_prec[l])) return fail(MG_ERR_PREC, "level_prec[%d] is not a format", l);
            prec[l] = (int)level_prec[l];
        }
    mg_ctx *h = new mg_ctx();
    h->batched = true;
    h->dim = 3;
    h->opt = o;
    h->Lmax = Lmax;
    h->bprec = prec;
    h->inst.resize(ninst);
    size_t off = 0;
    int parts = 0;
    for (int i = 0; i < ninst; ++i) {
        auto &I = h->inst[i];
        I.n = n[i];
        const int copies = (int)std::count(n, n + ninst, n[i]);
        int m = 0;
        while ((1 << m) < n[i] + 1) ++m;
        I.nl = m;
        I.lv.resize(m);
        int nn = n[i];
        for (int l = 0; l < m; ++l) {
            LevelPlan &L = I.lv[l];
            L.n = nn, L.P = nn + 1;
            L.prec = l == m - 1 ? prec[Lmax - 1] : prec[l];
            L.elems = level_elems(3, L.P);
            const size_t bytes = align_up(L.elems * prec_bytes(L.prec), 256);
            L.off_b = off, off += bytes;
            L.off_c[0] = off, off += bytes;
            L.off_c[1] = off, off += bytes;
            if (nn > 1) {
                L.shs[SH_SMOOTH] = L.shs[SH_SWEEP] = L.shs[SH_PROLONG] = batched_shape(L.P, L.prec, copies);
                L.rsh = batched_rshape(L.P, L.prec, copies);
            }
            nn = (nn - 1) / 2;
        }
        {
            std::vector<int> ns(m), pr(m);
            for (int l = 0; l < m; ++l) ns[l] = I.lv[l].n, pr[l] = I.lv[l].prec;
            (void)alpha_code(3, ns, pr, std::vector<bool>(m, false), o.residual_scaling, &I.ascale);
        }
        const size_t fin = align_up(I.lv[0].elems * sizeof(double), 256);
        I.off_R = off, off += fin;
        I.off_U = off, off += fin;
        I.osh = batched_shape(I.lv[0].P, P_F64, copies);  // V = 4: FP64 rows
        I.part_off = parts;
        I.parts = std::max(stencil_blocks(3, I.lv[0].P, I.osh), flat_blocks(points(3, n[i])));
        parts += I.parts;
    }
    h->max_parts = parts;
    h->off_part = off, off += align_up((size_t)parts * 2 * sizeof(double), 256);
    h->off_scal_all = off, off += align_up((size_t)ninst * 4 * sizeof(double), 256);
    h->off_active = off, off += align_up((size_t)ninst * sizeof(int), 256);
    h->off_bmeta = off;
    build_batched_plan(h, nullptr);
    // room for the plans of other launch shapes (the autotuner's candidates
    // with shorter plane chunks have more work items)
    h->bmeta_cap = align_up(4 * h->bmeta_bytes, 256);
    off += h->bmeta_cap;
    h->ws_need = off;
    h->nl = Lmax;
    h->n = n[0];
    *out = h;
    return MG_OK;
}

mg_status_t ir_solve_batched(mg_handle h, const double *const *b, double *const *u, mg_stats_t *stats,
                             void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!h) return fail(MG_ERR_ARG, "null handle");
    if (!h->batched) return fail(MG_ERR_STATE, "ir_solve_batched needs a handle from mg_setup_batched");
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!b || !u) return fail(MG_ERR_ARG, "null argument");
    const int ni = (int)h->inst.size();
    for (int i = 0; i < ni; ++i)
        if (!b[i] || !u[i]) return fail(MG_ERR_ARG, "null pointer for instance %d", i);
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part_base = reinterpret_cast<double *>(h->ws + h->off_part);
    double *scal_all = reinterpret_cast<double *>(h->ws + h->off_scal_all);
    int *act_dev = reinterpret_cast<int *>(h->ws + h->off_active);
    const double *hs = h->host_scal_all;
    // per instance: ACTIVE (stepping), CHECK (recursive residual below tolerance,
    // to be confirmed from u), DONE (u written), STOP (failed, u still to be
    // written), DEAD (failed before any step; u untouched)
    enum { ACTIVE, CHECK, DONE, STOP, DEAD };
    std::vector<double> nb(ni, 0.0), rel(ni, 0.0);
    std::vector<int> k(ni, 0), state(ni, ACTIVE);
    std::vector<mg_status_t> st_i(ni, MG_OK);
    auto hist = [&](int i, int kk, double v) {
        if (stats && stats[i].history && kk < stats[i].history_cap) stats[i].history[kk] = v;
    };
    auto readback = [&]() -> mg_status_t {
        HIPCHK(hipMemcpyAsync(h->host_scal_all, scal_all, 4 * sizeof(double) * ni, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return MG_OK;
    };
    // r = b - A u of instance i into R (and u copied out to uout) with its norms;
    // with use_u == false, r = b
    auto resid = [&](int i, bool use_u, double *uout) -> hipError_t {
        const auto &I = h->inst[i];
        const LevelPlan &L = I.lv[0];
        const double hh = 1.0 / (double)(L.n + 1);
        double *part = part_base + 2 * (size_t)I.part_off;
        hipError_t e = launch_resid_flat(3, L.n, L.P, b[i], use_u ? (const double *)(h->ws + I.off_U) : nullptr,
                                         reinterpret_cast<double *>(h->ws + I.off_R), uout, 1.0 / (hh * hh), part, st);
        if (e == hipSuccess) e = launch_finalize(part, flat_blocks(points(3, L.n)), scal_all + 4 * i, I.ascale, st);
        return e;
    };
    // ||b||_2 of every instance, and the initial residual
    for (int i = 0; i < ni; ++i) {
        const auto &I = h->inst[i];
        if (h->opt.use_initial_guess) {
            HIPCHK(launch_resid_flat(3, I.n, I.lv[0].P, b[i], nullptr, nullptr, nullptr, 1.0,
                                     part_base + 2 * (size_t)I.part_off, st));
            HIPCHK(launch_finalize(part_base + 2 * (size_t)I.part_off, flat_blocks(points(3, I.n)), scal_all + 4 * i,
                                   I.ascale, st));
        } else {
            HIPCHK(resid(i, false, nullptr));
            HIPCHK(launch_fill_zero(h->ws + I.off_U, align_up(I.lv[0].elems * sizeof(double), 16), st));
        }
    }
    if ((s = readback()) != MG_OK) return s;
    bool any_guess = false;
    for (int i = 0; i < ni; ++i) {
        nb[i] = hs[4 * i + 2];
        if (!std::isfinite(nb[i])) {
            state[i] = DEAD, st_i[i] = MG_ERR_NONFINITE, rel[i] = NAN;
        } else if (nb[i] == 0.0) {
            HIPCHK(hipMemsetAsync(u[i], 0, sizeof(double) * points(3, h->inst[i].n), st));
            state[i] = DONE;
            hist(i, 0, 0.0);
        } else if (h->opt.use_initial_guess) {
            const auto &I = h->inst[i];
            HIPCHK(launch_pack(3, P_F64, P_F64, I.n, I.lv[0].P, u[i], h->ws + I.off_U, st));
            HIPCHK(resid(i, true, nullptr));
            any_guess = true;
        }
    }
    if (any_guess && (s = readback()) != MG_OK) return s;
    const bool graph = h->opt.use_graph && !h->prof;
    if (graph && !h->gexec) {
        if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enq_batched_step(h, h->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(MG_ERR_HIP, "capture of the batched step failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        h->graph = g;
        HIPCHK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    }
    for (;;) {
        // classify the stepping instances on their latest residual norms
        int nact = 0, ncheck = 0;
        for (int i = 0; i < ni; ++i) {
            if (state[i] != ACTIVE) continue;
            const double rn = hs[4 * i + 2];
            rel[i] = rn / nb[i];
            hist(i, k[i], rel[i]);
            if (!std::isfinite(rn)) {
                state[i] = STOP, st_i[i] = MG_ERR_NONFINITE;
            } else if (rn <= h->opt.rtol * nb[i]) {
                // a residual that was updated recursively is confirmed from u
                state[i] = k[i] > 0 ? CHECK : STOP;
                ncheck += k[i] > 0;
            } else if (k[i] >= h->opt.max_iter) {
                state[i] = STOP, st_i[i] = MG_ERR_NOT_CONVERGED;
            } else {
                ++nact;
            }
        }
        if (ncheck > 0) {
            for (int i = 0; i < ni; ++i)
                if (state[i] == CHECK) HIPCHK(resid(i, true, u[i]));
            if ((s = readback()) != MG_OK) return s;
            for (int i = 0; i < ni; ++i) {
                if (state[i] != CHECK) continue;
                const double rn = hs[4 * i + 2];
                rel[i] = rn / nb[i];
                hist(i, k[i], rel[i]);
                if (rn <= h->opt.rtol * nb[i]) {
                    state[i] = DONE;
                } else if (!std::isfinite(rn) || k[i] >= h->opt.max_iter) {
                    state[i] = DONE;  // u and rel already hold the final values
                    st_i[i] = std::isfinite(rn) ? MG_ERR_NOT_CONVERGED : MG_ERR_NONFINITE;
                } else {
                    state[i] = ACTIVE;  // continue from the true residual
                    ++nact;
                }
            }
        }
        if (nact == 0) break;
        for (int i = 0; i < ni; ++i) h->host_active[i] = state[i] == ACTIVE;
        HIPCHK(hipMemcpyAsync(act_dev, h->host_active, sizeof(int) * ni, hipMemcpyHostToDevice, st));
        if (graph) {
            HIPCHK(hipGraphLaunch(h->gexec, st));
        } else {
            hipError_t e = enq_batched_step(h, st);
            if (e != hipSuccess) return fail(MG_ERR_HIP, "batched step failed: %s", hipGetErrorString(e));
        }
        HIPCHK(hipStreamSynchronize(st));
        for (int i = 0; i < ni; ++i)
            if (state[i] == ACTIVE) ++k[i];
    }
    // instances that stopped without a confirmation: true residual and u
    bool pending = false;
    for (int i = 0; i < ni; ++i)
        if (state[i] == STOP) {
            HIPCHK(resid(i, true, u[i]));
            pending = true;
        }
    if (pending) {
        if ((s = readback()) != MG_OK) return s;
        for (int i = 0; i < ni; ++i)
            if (state[i] == STOP) rel[i] = hs[4 * i + 2] / nb[i];
    }
    HIPCHK(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    mg_status_t result = MG_OK;
    int first_bad = -1;
    for (int i = 0; i < ni; ++i) {
        if (stats) {
            stats[i].iterations = k[i];
            stats[i].rel_residual = nb[i] == 0.0 ? 0.0 : rel[i];
            stats[i].seconds = secs;
        }
        if (st_i[i] != MG_OK && result == MG_OK) result = st_i[i], first_bad = i;
    }
    if (result != MG_OK) return fail(result, "%s (first in instance %d)", mg_status_string(result), first_bad);
    return MG_OK;
}

mg_status_t mg_instances(mg_handle h, int *ninst) {
    if (!h || !ninst) return fail(MG_ERR_ARG, "null argument");
    *ninst = h->batched ? (int)h->inst.size() : 1;
    return MG_OK;
}

}  // extern "C"

// ============================================================================
// Many right-hand sides, interleaved
// ============================================================================
namespace {

int m_zc(int prec, int P, int K) {
    const long per_chunk = (long)(P - 1) * (K / m_vec(prec)) * (P - 1);
    const long nch = std::max(1L, ((1L << 19) + per_chunk - 1) / per_chunk);
    return std::max(1, std::min((int)((P - 1 + nch - 1) / nch), 64));
}

hipError_t enq_multi_step(mg_ctx *h, hipStream_t st) {
    const int K = h->nrhs, nl = h->nl;
    const bool alias = finest_alias(h);
    double *sc = scal(h);
    const int *act = at_ws<int>(h, h->off_act);
    auto rhs = [&](int l) -> const void * { return (l == 0 && alias) ? (const void *)Rbuf(h) : bbuf(h, l); };
    for (int l = 0; l + 1 < nl; ++l) {
        LevelPlan &L = h->lv[l];
        const double N = (double)points(3, L.n) * K;
        const double s = sb(L.prec);
        MArgs a;
        a.prec = L.prec, a.P = L.P, a.K = K, a.zc = L.shs[SH_SMOOTH].zc, a.omega = h->opt.omega;
        a.cout = cbuf(h, l, 0);
        if (l == 0 && !alias) {
            a.r = Rbuf(h), a.inv = sc + K, a.act = act, a.bout = bbuf(h, 0);
            RUN(h, st, "smooth2_scaled", l, N * (8 + 2 * s), launch_m_stage(MS_SMOOTH2, a, st));
        } else {
            a.b = rhs(l);
            RUN(h, st, "smooth2", l, N * 2 * s, launch_m_stage(MS_SMOOTH2, a, st));
        }
        int cur = 0;
        for (int k = 2; k < h->opt.nu1; ++k) {
            MArgs w;
            w.prec = L.prec, w.P = L.P, w.K = K, w.zc = L.shs[SH_SWEEP].zc, w.omega = h->opt.omega;
            w.b = rhs(l), w.cin = cbuf(h, l, cur), w.cout = cbuf(h, l, cur ^ 1);
            RUN(h, st, "sweep", l, N * 3 * s, launch_m_stage(MS_SWEEP, w, st));
            cur ^= 1;
        }
        h->cur[l] = cur;
        MArgs r;
        r.prec = L.prec, r.pc = h->lv[l + 1].prec, r.P = L.P, r.K = K, r.zc = L.shs[SH_SWEEP].zc;
        r.b = rhs(l), r.cin = cbuf(h, l, cur), r.cout = bbuf(h, l + 1);
        RUN(h, st, "resid_restrict", l, N * 2 * s + (double)points(3, h->lv[l + 1].n) * K * sb(r.pc),
            launch_m_restrict2(r, h->ws + h->off_mres, L.rsh.zcc, st));
    }
    RUN(h, st, "coarse_solve", nl - 1, 2.0 * K * sb(h->lv[nl - 1].prec),
        launch_m_coarse(h->lv[nl - 1].prec, K, bbuf(h, nl - 1), cbuf(h, nl - 1, 0), st));
    h->cur[nl - 1] = 0;
    for (int l = nl - 2; l >= 0; --l) {
        LevelPlan &L = h->lv[l];
        const double N = (double)points(3, L.n) * K;
        const double s = sb(L.prec);
        int cur = h->cur[l];
        MArgs a;
        a.prec = L.prec, a.pc = h->lv[l + 1].prec, a.P = L.P, a.K = K, a.zc = L.shs[SH_PROLONG].zc;
        a.omega = h->opt.omega;
        a.b = rhs(l), a.cin = cbuf(h, l, cur), a.ec = cbuf(h, l + 1, h->cur[l + 1]), a.cout = cbuf(h, l, cur ^ 1);
        RUN(h, st, "prolong", l, N * 2 * s + (double)points(3, h->lv[l + 1].n) * K * sb(a.pc),
            launch_m_prolong_field(a, st));
        RUN(h, st, "prolong_sweep", l, N * 3 * s, launch_m_stage(MS_SWEEP, a, st));
        cur ^= 1;
        for (int k = 1; k < h->opt.nu2; ++k) {
            MArgs w;
            w.prec = L.prec, w.P = L.P, w.K = K, w.zc = L.shs[SH_SWEEP].zc, w.omega = h->opt.omega;
            w.b = rhs(l), w.cin = cbuf(h, l, cur), w.cout = cbuf(h, l, cur ^ 1);
            RUN(h, st, "sweep", l, N * 3 * s, launch_m_stage(MS_SWEEP, w, st));
            cur ^= 1;
        }
        h->cur[l] = cur;
    }
    LevelPlan &L = h->lv[0];
    const double hh = 1.0 / (double)(L.n + 1);
    const double N = (double)points(3, L.n) * K;
    MArgs u;
    u.prec = L.prec, u.P = L.P, u.K = K, u.zc = L.osh.zc, u.cin = cbuf(h, 0, h->cur[0]), u.act = act;
    RUN(h, st, "ir_update", 0, N * (32 + sb(L.prec)), launch_m_update(u, Rbuf(h), Ubuf(h), sc, hh * hh, part(h), st));
    RUN(h, st, "norm_finalize", 0, 16.0 * h->m_upd_blocks * K,
        launch_m_finalize(part(h), h->m_upd_blocks, K, sc, act, h->ascale, st));
    return hipMemcpyAsync(h->host_scal_m, sc, 4 * sizeof(double) * K, hipMemcpyDeviceToHost, st);
}

// ---- many-right-hand-side autotuner --------------------------------------------
// Per level, the planes per thread of the first smoothing, the sweeps (and the
// residual pass of the restriction), the prolongation and the coarse planes
// per block of the restriction, each timed as a whole refinement step with
// every column active (the update keeps its shape: its block count sizes the
// reduction partials).  Every choice forms the same roundings.
std::string multi_tune_key(const mg_ctx *h) {
    const std::string dk = device_key();
    if (dk.empty()) return dk;
    std::string k = dk + "|multi|n" + std::to_string(h->n) + "|K" + std::to_string(h->nrhs) + "|nu" +
                    std::to_string(h->opt.nu1) + "," + std::to_string(h->opt.nu2) + "|sc" +
                    std::to_string(h->opt.residual_scaling) + "|p";
    for (int l = 0; l < h->nl; ++l) k += std::to_string(h->lv[l].prec);
    return k;
}

constexpr int kMLevelInts = 4;  // zc of smoothing, sweeps, prolongation; zcc of the restriction

bool apply_multi_state(mg_ctx *h, const std::vector<int> &v) {
    if (v.size() != (size_t)(h->nl - 1) * kMLevelInts) return false;
    for (int l = 0; l + 1 < h->nl; ++l) {
        const int *q = v.data() + l * kMLevelInts, P = h->lv[l].P;
        for (int j = 0; j < 3; ++j)
            if (q[j] < 1 || q[j] > std::max(1, P - 1)) return false;
        if (q[3] < 1 || q[3] > std::max(1, P / 2 - 1)) return false;
    }
    for (int l = 0; l + 1 < h->nl; ++l) {
        const int *q = v.data() + l * kMLevelInts;
        LevelPlan &L = h->lv[l];
        L.shs[SH_SMOOTH].zc = q[0], L.shs[SH_SWEEP].zc = q[1], L.shs[SH_PROLONG].zc = q[2], L.rsh.zcc = q[3];
    }
    return true;
}

mg_status_t autotune_multi(mg_ctx *h, hipStream_t st) {
    const std::string key = multi_tune_key(h);
    std::vector<int> v;
    if (cache_read(key, v) && apply_multi_state(h, v)) return MG_OK;
    const int K = h->nrhs;
    for (int k = 0; k < K; ++k) h->host_mask[k] = 1;
    HIPCHK(hipMemcpy(h->ws + h->off_act, h->host_mask, sizeof(int) * K, hipMemcpyHostToDevice));
    auto step_ms = [&]() { return time_ms(st, [&]() { return enq_multi_step(h, st); }, 2); };
    v.clear();
    for (int l = 0; l + 1 < h->nl; ++l) {
        LevelPlan &L = h->lv[l];
        int *knobs[4] = {&L.shs[SH_SMOOTH].zc, &L.shs[SH_SWEEP].zc, &L.shs[SH_PROLONG].zc, &L.rsh.zcc};
        const int lim[4] = {L.P - 1, L.P - 1, L.P - 1, L.P / 2 - 1};
        for (int j = 0; j < 4; ++j) {
            if (lim[j] < 2) continue;
            int bestv = *knobs[j];
            float best = step_ms();
            for (int zc : {1, 2, 4, 8, 16, 32, 64}) {
                if (zc > lim[j] || zc == bestv) continue;
                *knobs[j] = zc;
                const float t = step_ms();
                if (t < best) best = t, bestv = zc;
            }
            *knobs[j] = bestv;
        }
        v.insert(v.end(), {L.shs[SH_SMOOTH].zc, L.shs[SH_SWEEP].zc, L.shs[SH_PROLONG].zc, L.rsh.zcc});
    }
    HIPCHK(hipMemsetAsync(h->ws, 0, h->ws_need, st));
    HIPCHK(hipStreamSynchronize(st));
    cache_write(key, v);
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status_t mg_setup_multi(mg_handle *out, int dim, int n, int nrhs, const mg_prec_t *level_prec,
                           const mg_options_t *opt) {
    if (!out) return fail(MG_ERR_ARG, "null argument");
    if (dim != 3) return fail(MG_ERR_SHAPE, "many right-hand sides are 3-D (dim = 3)");
    if (n < 3 || n > 511 || ((n + 1) & n) != 0) return fail(MG_ERR_SHAPE, "n must be 2^m - 1 with 2 <= m <= 9, got %d", n);
    if (nrhs < 4 || nrhs > 64 || (nrhs & (nrhs - 1)))
        return fail(MG_ERR_ARG, "nrhs must be 4, 8, 16, 32 or 64 (got %d)", nrhs);
    mg_options_t o;
    mg_default_options(&o);
    if (opt) o = *opt;
    if (o.rescale_half) return fail(MG_ERR_ARG, "rescale_half is only available on single-grid handles");
    if (o.defer_update) return fail(MG_ERR_ARG, "defer_update is only available on single-grid handles");
    if (o.discretization != MG_DISC_FD)
        return fail(MG_ERR_ARG, "the Q1 discretisation is only available on single-grid handles");
    if (o.cycles_per_step != 1)
        return fail(MG_ERR_ARG, "cycles_per_step other than 1 is only available on single-grid handles");
    if (o.nu1 < 2 || o.nu1 > 16 || o.nu2 < 1 || o.nu2 > 16)
        return fail(MG_ERR_ARG, "many right-hand sides need 2 <= nu1 <= 16 and 1 <= nu2 <= 16");
    if (!(o.omega > 0.0 && o.omega < 2.0) || o.max_iter < 0 || !(o.rtol >= 0.0)) return fail(MG_ERR_ARG, "bad options");
    int m = 0;
    while ((1 << m) < n + 1) ++m;
    std::vector<int> prec(m, P_F64);
    if (level_prec)
        for (int l = 0; l < m; ++l) {
            if (!valid_prec((int)level_prec[l])) return fail(MG_ERR_PREC, "level_prec[%d] is not a format", l);
            prec[l] = (int)level_prec[l];
        }
    for (int l = 0; l < m; ++l)
        if (!m_supported(prec[l], nrhs))
            return fail(MG_ERR_ARG, "nrhs = %d is below the %d columns a thread of level %d handles", nrhs,
                        m_vec(prec[l]), l);
    int ascale = 0;
    {
        std::vector<int> ns(m);
        for (int l = 0, nn = n; l < m; ++l, nn = (nn - 1) / 2) ns[l] = nn;
        (void)alpha_code(3, ns, prec, std::vector<bool>(m, false), o.residual_scaling, &ascale);
    }
    mg_ctx *h = new mg_ctx();
    h->dim = 3, h->n = n, h->nl = m, h->opt = o, h->nrhs = nrhs;
    h->ascale = ascale;
    h->lv.resize(m);
    const int K = nrhs;
    size_t off = 0;
    int nn = n;
    for (int l = 0; l < m; ++l) {
        LevelPlan &L = h->lv[l];
        L.n = nn, L.P = nn + 1, L.prec = prec[l];
        L.elems = level_elems(3, L.P) * K;
        const size_t bytes = align_up(L.elems * prec_bytes(L.prec), 256);
        L.off_b = off, off += bytes;
        L.off_c[0] = off, off += bytes;
        L.off_c[1] = off, off += bytes;
        if (nn > 1) {
            Shape s{m_vec(L.prec), m_zc(L.prec, L.P, K), 256, 0, 0};
            L.shs[SH_SMOOTH] = L.shs[SH_SWEEP] = L.shs[SH_PROLONG] = s;
            L.osh = Shape{4, m_zc(P_F64, L.P, K), 256, 0, 0};
            L.rsh = RShape{m_vec(L.prec), 1, m_zc(L.prec, L.P / 2, K), 0};
        }
        nn = (nn - 1) / 2;
    }
    const size_t fin = align_up(h->lv[0].elems * sizeof(double), 256);
    h->off_R = off, off += fin;
    h->off_U = off, off += fin;
    h->m_upd_blocks = m_update_blocks(h->lv[0].prec, h->lv[0].P, K, h->lv[0].osh.zc);
    h->max_parts = std::max(h->m_upd_blocks, m_resid_blocks(n));
    h->off_part = off, off += align_up((size_t)h->max_parts * K * 2 * sizeof(double), 256);
    h->off_scal = off, off += align_up(4 * sizeof(double) * K, 256);
    h->off_act = off, off += 256;
    h->off_mask = off, off += 256;
    h->off_zmask = off, off += 256;
    size_t mres = 0;
    for (int l = 0; l + 1 < m; ++l) mres = std::max(mres, m_resid_bytes(h->lv[l].prec, h->lv[l].elems));
    h->off_mres = off, off += align_up(mres, 256);
    h->ws_need = off;
    *out = h;
    return MG_OK;
}

mg_status_t ir_solve_multi(mg_handle h, const double *b, double *u, mg_stats_t *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!h) return fail(MG_ERR_ARG, "null handle");
    if (!h->nrhs) return fail(MG_ERR_STATE, "ir_solve_multi needs a handle from mg_setup_multi");
    mg_status_t s = need_ws(h);
    if (s != MG_OK) return s;
    if (!b || !u) return fail(MG_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int K = h->nrhs;
    const LevelPlan &L = h->lv[0];
    const int n = L.n, P = L.P;
    const double hh = 1.0 / (double)(n + 1);
    const double inv_h2 = 1.0 / (hh * hh);
    const int scaling = h->ascale;
    const int rparts = m_resid_blocks(n);
    double *sc = scal(h);
    const double *hs = h->host_scal_m;
    int *act_dev = at_ws<int>(h, h->off_act);
    int *mask_dev = at_ws<int>(h, h->off_mask);
    const int *zmask = at_ws<int>(h, h->off_zmask);
    int *hact = h->host_mask, *hmask = h->host_mask + K;
    enum { ACTIVE, CHECK, DONE, STOP, DEAD };
    std::vector<double> nb(K, 0.0), rel(K, 0.0);
    std::vector<int> it(K, 0), state(K, ACTIVE);
    std::vector<mg_status_t> st_k(K, MG_OK);
    auto hist = [&](int k, int kk, double v) {
        if (stats && stats[k].history && kk < stats[k].history_cap) stats[k].history[kk] = v;
    };
    auto readback = [&]() -> mg_status_t {
        HIPCHK(hipMemcpyAsync(h->host_scal_m, sc, 4 * sizeof(double) * K, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return MG_OK;
    };
    // true residual and norms of the columns in `which` (mask uploaded first)
    auto resid_cols = [&](const std::vector<int> &which) -> mg_status_t {
        HIPCHK(hipStreamSynchronize(st));  // an earlier copy may still read hmask
        for (int k = 0; k < K; ++k) hmask[k] = which[k];
        HIPCHK(hipMemcpyAsync(mask_dev, hmask, sizeof(int) * K, hipMemcpyHostToDevice, st));
        HIPCHK(launch_m_resid(n, P, K, b, Ubuf(h), Rbuf(h), nullptr, mask_dev, inv_h2, part(h), st));
        HIPCHK(launch_m_finalize(part(h), rparts, K, sc, mask_dev, scaling, st));
        return readback();
    };
    // ||b||_2 per column (r = b when starting from zero)
    if (h->opt.use_initial_guess) {
        HIPCHK(launch_m_resid(n, P, K, b, nullptr, nullptr, nullptr, nullptr, inv_h2, part(h), st));
    } else {
        HIPCHK(launch_m_resid(n, P, K, b, nullptr, Rbuf(h), nullptr, nullptr, inv_h2, part(h), st));
        HIPCHK(launch_fill_zero(Ubuf(h), align_up(L.elems * sizeof(double), 16), st));
    }
    HIPCHK(launch_m_finalize(part(h), rparts, K, sc, nullptr, scaling, st));
    if ((s = readback()) != MG_OK) return s;
    for (int k = 0; k < K; ++k) {
        nb[k] = hs[2 * K + k];
        if (!std::isfinite(nb[k])) {
            state[k] = DEAD, st_k[k] = MG_ERR_NONFINITE, rel[k] = NAN;
        } else if (nb[k] == 0.0) {
            state[k] = DONE;  // u = 0: its column of U is (made) zero
            hist(k, 0, 0.0);
        }
    }
    if (h->opt.use_initial_guess) {
        for (int k = 0; k < K; ++k) hmask[k] = nb[k] != 0.0;
        HIPCHK(hipMemcpyAsync(mask_dev, hmask, sizeof(int) * K, hipMemcpyHostToDevice, st));
        HIPCHK(launch_m_pack(n, P, K, u, Ubuf(h), mask_dev, st));
        std::vector<int> all(K, 1);
        if ((s = resid_cols(all)) != MG_OK) return s;
    }
    const bool graph = h->opt.use_graph && !h->prof;
    if (graph && !h->gexec) {
        if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enq_multi_step(h, h->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(MG_ERR_HIP, "capture of the interleaved step failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        h->graph = g;
        HIPCHK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    }
    for (;;) {
        int nact = 0, ncheck = 0;
        std::vector<int> check(K, 0);
        for (int k = 0; k < K; ++k) {
            if (state[k] != ACTIVE) continue;
            const double rn = hs[2 * K + k];
            rel[k] = rn / nb[k];
            hist(k, it[k], rel[k]);
            if (!std::isfinite(rn)) {
                state[k] = STOP, st_k[k] = MG_ERR_NONFINITE;
            } else if (rn <= h->opt.rtol * nb[k]) {
                state[k] = it[k] > 0 ? CHECK : STOP;
                if (it[k] > 0) check[k] = 1, ++ncheck;
            } else if (it[k] >= h->opt.max_iter) {
                state[k] = STOP, st_k[k] = MG_ERR_NOT_CONVERGED;
            } else {
                ++nact;
            }
        }
        if (ncheck > 0) {
            // confirm from u; only these columns' R and norms are rewritten
            if ((s = resid_cols(check)) != MG_OK) return s;
            for (int k = 0; k < K; ++k) {
                if (!check[k]) continue;
                const double rn = hs[2 * K + k];
                rel[k] = rn / nb[k];
                hist(k, it[k], rel[k]);
                if (rn <= h->opt.rtol * nb[k]) {
                    state[k] = DONE;
                } else if (!std::isfinite(rn) || it[k] >= h->opt.max_iter) {
                    state[k] = DONE;
                    st_k[k] = std::isfinite(rn) ? MG_ERR_NOT_CONVERGED : MG_ERR_NONFINITE;
                } else {
                    state[k] = ACTIVE;
                    ++nact;
                }
            }
        }
        if (nact == 0) break;
        for (int k = 0; k < K; ++k) hact[k] = state[k] == ACTIVE;
        HIPCHK(hipMemcpyAsync(act_dev, hact, sizeof(int) * K, hipMemcpyHostToDevice, st));
        if (graph) {
            HIPCHK(hipGraphLaunch(h->gexec, st));
        } else {
            hipError_t e = enq_multi_step(h, st);
            if (e != hipSuccess) return fail(MG_ERR_HIP, "interleaved step failed: %s", hipGetErrorString(e));
        }
        HIPCHK(hipStreamSynchronize(st));
        for (int k = 0; k < K; ++k)
            if (state[k] == ACTIVE) ++it[k];
    }
    std::vector<int> stop(K, 0);
    bool any_stop = false;
    for (int k = 0; k < K; ++k)
        if (state[k] == STOP) stop[k] = 1, any_stop = true;
    if (any_stop) {
        if ((s = resid_cols(stop)) != MG_OK) return s;
        for (int k = 0; k < K; ++k)
            if (stop[k]) rel[k] = hs[2 * K + k] / nb[k];
    }
    // u out, every column (held columns keep their last iterate)
    HIPCHK(launch_m_resid(n, P, K, b, Ubuf(h), nullptr, u, zmask, inv_h2, part(h), st));
    HIPCHK(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    mg_status_t result = MG_OK;
    int first_bad = -1;
    for (int k = 0; k < K; ++k) {
        if (stats) {
            stats[k].iterations = it[k];
            stats[k].rel_residual = nb[k] == 0.0 ? 0.0 : rel[k];
            stats[k].seconds = secs;
        }
        if (st_k[k] != MG_OK && result == MG_OK) result = st_k[k], first_bad = k;
    }
    if (result != MG_OK) return fail(result, "%s (first in right-hand side %d)", mg_status_string(result), first_bad);
    return MG_OK;
}

mg_status_t mg_rhs_count(mg_handle h, int *nrhs) {
    if (!h || !nrhs) return fail(MG_ERR_ARG, "null argument");
    *nrhs = h->nrhs ? h->nrhs : 1;
    return MG_OK;
}

}  // extern "C"
