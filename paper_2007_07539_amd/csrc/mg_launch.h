// Host-side launch interface of the gfx950 multigrid kernels (internal to the
// library; the public ABI is include/mgir.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "mgir.h"

namespace mg {

enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

inline size_t prec_bytes(int p) { return p == P_F64 ? 8 : p == P_F32 ? 4 : 2; }

// Launch shape of one z-marching stencil kernel.
struct Shape {
    int V;    // elements per thread along x (4 or 8), V <= P
    int zc;   // planes (3-D) or rows (2-D) marched by one thread
    int bs;   // threads per block (multiple of 64, <= 256), register-queue kernel only
    int xcd;  // 1: remap block ids so consecutive tiles share an XCD
    int ty;   // 3-D only: > 0 selects the LDS-plane kernel with ty output rows per block
    int dp = 1;  // LDS-plane kernel: planes loaded ahead of the one being computed (1 or 2)
    int sg = 1;  // LDS-plane prolongation: 1 = stage the z-interpolated coarse plane in LDS
                 // where it fits, 0 = every row reads its coarse rows from memory
};

// LDS bytes of the LDS-plane kernel for a level of storage size sb bytes.
inline size_t march_lds_bytes(int P, int ty, size_t sb) { return 2 * (size_t)(ty + 2) * P * sb; }

// Launch shape of the residual + restriction kernel.
struct RShape {
    int V;     // fine elements per thread along x (4 or 8); the coarse side uses V/2
    int tyc;   // coarse rows per block (3-D)
    int zcc;   // coarse planes (3-D) or rows (2-D) per block
    int pipe;  // 3-D only: 1 selects the pipelined kernel (correction plane in LDS)
};

// Elements of a padded level array: (P + 2) planes of P*P (3-D) or (P + 2)
// rows of P (2-D).
inline size_t level_elems(int D, int P) { return D == 3 ? (size_t)(P + 2) * P * P : (size_t)(P + 2) * P; }

// Number of blocks a stencil launch uses (= reduction partials it writes).
int stencil_blocks(int D, int P, const Shape &s);
int restrict_blocks(int D, int P, const RShape &s);
size_t restrict_lds_bytes(int D, int P, int pf, const RShape &s);
int flat_blocks(long N);

// Pre-smoothing from zero: c = S^2(0) (two fused sweeps) or S(0) when
// two == false.  The right-hand side is b (level format) or, when r != NULL,
// b = round(r * scal[1]) from the FP64 residual r, which is then also written
// to b_out (fused scale-and-cast of the refinement loop).
hipError_t launch_smooth_first(int D, int prec, int P, const void *b, const double *r, const double *scal,
                               void *b_out, void *c, double omega, bool two, const Shape &s,
                               hipStream_t st);
// One damped-Jacobi sweep: c_out = c + k (b - L c).
hipError_t launch_sweep(int D, int prec, int P, const void *b, const void *c, void *c_out, double omega,
                        const Shape &s, hipStream_t st);
// b_c = round(FW(b - L c)) onto the coarse level.
hipError_t launch_restrict(int D, int pf, int pc, int P, const void *b, const void *c, void *bc,
                           const RShape &s, hipStream_t st);
// c_out = S(round(c + 4 P e_c)) when sweep, else round(c + 4 P e_c).
hipError_t launch_prolong(int D, int pf, int pc, int P, const void *c, const void *ec, const void *b,
                          void *c_out, double omega, bool sweep, const Shape &s, hipStream_t st);
// Base level (n = 1): c = b / (2D).
hipError_t launch_coarse(int D, int prec, const void *b, void *c, hipStream_t st);
// Refinement update of Algorithm 2 (solution and residual update), FP64: U += a h^2 c, R -= a L c,
// with a = scal[0]; writes one (sum r^2, max |r|) pair per block to part.
hipError_t launch_outer_update(int D, int prec, int P, const void *c, double *R, double *U,
                               const double *scal, double h2, double *part, const Shape &s,
                               hipStream_t st);
// Dense-index pass: r = b - A U (or r = b when U == NULL), optionally stored
// to the padded R and U copied out to the dense uout; (sum r^2, max |r|)
// partials per block.
hipError_t launch_resid_flat(int D, int n, int P, const double *b, const double *U, double *R,
                             double *uout, double inv_h2, double *part, hipStream_t st);
// Reduce partials: scal = {alpha, 1/alpha, ||r||_2, ||r||_inf}.  scaling 0:
// alpha = 1; scaling 1 + j: alpha = 2^j ||r||_inf (also for launch_m_finalize).
// A non-null ctr is incremented (the slot counter of postponed updates).
hipError_t launch_finalize(const double *part, int nparts, double *scal, int scaling, hipStream_t st,
                           int *ctr = nullptr);
// Dense <-> padded copies with format conversion (round to nearest even).
hipError_t launch_pack(int D, int src_prec, int dst_prec, int n, int P, const void *src, void *dst,
                       hipStream_t st);
hipError_t launch_unpack(int D, int src_prec, int dst_prec, int n, int P, const void *src, void *dst,
                         hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
// Copy (kind 0), read (1) or write (2) `bytes` with 16-byte lanes.
hipError_t launch_probe(void *dst, const void *src, size_t bytes, int kind, int blocks, unsigned *sink,
                        hipStream_t st);

// Last post-smoothing sweep of the finest 3-D level fused with the refinement
// update (LDS-plane kernel; s.ty rows per block, s.V values per thread).
struct SweepUpdateArgs {
    const void *c = nullptr;    // correction before the sweep (level format)
    const void *b = nullptr;    // right-hand side (level format), or R: then b = round(R * scal[1]) is formed
    const double *R = nullptr;  // residual in
    double *Rout = nullptr;     // residual out: == R (in place) unless b == R, then another array
    double *U = nullptr;        // iterate, updated unless cdefer is set
    void *cdefer = nullptr;     // ring of postponed corrections (level format), or null
    const int *ctr = nullptr;   // ... slot of this step
    size_t cstride = 0;         // ... elements between slots
    double *adef = nullptr;     // ... alpha of each slot
    const double *scal = nullptr;
    double h2 = 0.0, omega = 0.8;
    double *part = nullptr;
};
size_t sweep_update_lds_bytes(int P, int ty, size_t sb);
bool sweep_update_ok(int P, int prec, const Shape &s);
int sweep_update_blocks(int P, const Shape &s);
// Lets the kernel's instances allocate up to kLdsMax of LDS (FP64 rows at
// P = 512 need more than 64 KB); call before the first launch, outside a
// stream capture.
hipError_t sweep_update_prepare();
hipError_t launch_sweep_update(int prec, int P, const SweepUpdateArgs &a, const Shape &s, hipStream_t st);
// Apply postponed corrections: U += adef[j] h^2 c_j for j = 0 .. count-1 in
// order (c_j at cdefer + j * cstride elements, level format prec; elems
// padded elements each), then *ctr = 0.
hipError_t launch_defer_flush(int prec, const void *cdefer, size_t cstride, const double *adef, int count, double h2,
                              double *U, size_t elems, int *ctr, hipStream_t st, bool from_zero = false);

// First pre-smoothing of the finest 3-D level from the FP64 residual (scaled
// and cast) fused with the residual + full-weighting restriction of its
// result; writes b = round(r / alpha), c2 and the coarse right-hand side.
// Levels with P/8 dividing 64 (FP64 ones: at most 512 threads and kLdsMax of
// LDS, one coarse row per tile at P = 512); s.tyc coarse rows and s.zcc
// coarse planes per block.
// LDS one workgroup may allocate on gfx950.
constexpr size_t kLdsMax = 160 * 1024;
// narrow: c1 and c2 in LDS in the level's 2-byte format (RShape pipe 4)
size_t smooth_restrict_lds_bytes(int P, int tyc, int prec, bool narrow);
// Lets every instance of the fused kernel allocate up to kLdsMax of LDS; call
// once per process before the first launch (not inside a stream capture).
hipError_t smooth_restrict_prepare();
bool smooth_restrict_ok(int P, int prec, const RShape &s);
hipError_t launch_smooth_restrict(int prec, int pc, int P, const double *R, const double *scal, void *bout,
                                  void *cout, void *bc, double omega, const RShape &s, hipStream_t st);
// The same from the level's stored right-hand side b (no b output).
hipError_t launch_smooth_restrict_b(int prec, int pc, int P, const void *b, void *cout, void *bc, double omega,
                                    const RShape &s, hipStream_t st);

// Residual rescaling on restriction into a half-precision level.  pa is the
// fine level's accumulator format (P_F64 or P_F32), prec the coarse level's
// (P_F16 or P_BF16); n counts padded elements.  part needs
// rescale_part_count() doubles; rs receives {s, 1/s}.
size_t rescale_part_count();
// CG base solve (base of n >= 2 points per dimension, level format prec,
// op 0: finite-difference stencil, 1: Q1);
// scratch holds x, r, p, q at cg_scratch_stride(prec, elems) bytes apart.
size_t cg_scratch_stride(int prec, size_t elems);
hipError_t launch_cg_base(int D, int prec, int n, int P, const void *b, void *c, void *scratch, size_t stride,
                          double tol, int max_iter, int op, hipStream_t st);

// Q1 finite elements (grid-scaled stencil S, see mg_q1.hip).  n is the level's
// interior size (odd for levels with a coarser one), P = n + 1.
// launch_q1_restrict writes the fine residual into rs (q1_resid_bytes) first.
// Launch shape of the LDS-staged Q1 sweep, residual and update (3-D levels
// stored in a 2-byte format, P a multiple of 4): ty rows per block, zc planes
// per chunk; {0, 0} is the built-in choice.  Other levels ignore it.  The
// residual runs fused with the restriction (even ty and zc) unless split = 1.
struct Q1Shape {
    int ty = 0, zc = 0;
    int split = 0;  // residual kernel: 1 = residual and restriction as two kernels
};
// Whether the level takes the LDS-staged kernels; whether s fits its kernel
// (0 sweep, 1 residual, 2 update: threads, LDS, at most flat_blocks(points)
// blocks where they write partials); the shape the kernel uses for s.
bool q1_lds_level(int D, int prec, int n, int P);
bool q1_shape_ok(int D, int prec, int n, int P, int kernel, const Q1Shape &s);
Q1Shape q1_shape_used(int D, int prec, int n, int P, int kernel, const Q1Shape &s);
size_t q1_resid_bytes(int D, int prec, int P);
int q1_outer_blocks(int D, int n, int prec, const Q1Shape &s = Q1Shape{});
hipError_t launch_q1_first(int D, int prec, int n, int P, const void *b, const double *R, const double *scal,
                           void *b_out, void *c_out, double omega, hipStream_t st);
hipError_t launch_q1_sweep(int D, int prec, int n, int P, const void *b, const void *c, void *c_out, double omega,
                           hipStream_t st, const Q1Shape &s = Q1Shape{});
hipError_t launch_q1_restrict(int D, int pf, int pc, int n, int P, const void *b, const void *c, void *rs, void *bc,
                              hipStream_t st, const Q1Shape &s = Q1Shape{});
// s: the shape of the sweep that follows the prolongation
hipError_t launch_q1_prolong(int D, int pf, int pc, int n, int P, const void *c, const void *ec, const void *b,
                             void *c_out, double omega, hipStream_t st, const Q1Shape &s = Q1Shape{});
// cdefer != nullptr: postponed update (the correction goes to ring slot *ctr
// of cstride elements, alpha to adef[*ctr]; U untouched).
hipError_t launch_q1_outer(int D, int prec, int n, int P, const void *c, double *R, double *U, const double *scal,
                           double f, double *part, hipStream_t st, void *cdefer = nullptr, size_t cstride = 0,
                           double *adef = nullptr, const int *ctr = nullptr, const Q1Shape &s = Q1Shape{});
hipError_t launch_q1_resid_flat(int D, int n, int P, const double *b, const double *U, double *R, double *uout,
                                double hd, double *part, hipStream_t st);
hipError_t launch_q1_coarse(int D, int prec, const void *b, void *c, hipStream_t st);
hipError_t launch_absmax(int pa, const void *t, long n, double *part, double *rs, hipStream_t st);
hipError_t launch_scale_cast(int pa, int prec, const void *t, const double *rs, void *out, long n, hipStream_t st);
hipError_t launch_scale_widen(int prec, int pa, const void *c, const double *rs, void *out, long n, hipStream_t st);

// Fused coarse end of a 3-D V-cycle in one workgroup (LDS-resident levels):
// nlev grids of format prec with pitches P0 = 4 * 2^(nlev-1), ..., 4, then the
// one-point base of format pb.  b: right-hand side of the first (padded, pitch
// P0); c: receives its corrected, post-smoothed correction.
size_t tail_lds_bytes(int prec, int pb, int P0, int nlev);  // 0 if unsupported
hipError_t launch_tail(int prec, int pb, int P0, int nlev, const void *b, void *c, int nu1, int nu2, double omega,
                       hipStream_t st);

// ---- batched instances -------------------------------------------------------
// Per-(instance, level) arguments of one batched launch.
struct BDesc {
    const void *b;       // right-hand side (level format); FP64 residual for the scaled first smoothing
    const void *cin;     // input correction (sweep, prolongation, update, restriction)
    void *cout;          // output correction; coarse right-hand side for the restriction
    const void *ec;      // coarse correction (prolongation)
    void *bout;          // scaled right-hand side written by the first smoothing
    const double *scal;  // alpha, 1/alpha, ||r||_2, ||r||_inf of the instance
    double *R, *U;       // FP64 residual and iterate (update)
    double h2;
    int P, zc, nchunks;  // stencil launch shape of this grid
    int tyc, zcc, ytiles;
    int part_off;        // first reduction partial of the instance (update)
    int inst;
    int ty;              // LDS-plane kernels: rows per block (ytiles = its y tiles)
};
struct BItem {
    int d, blk;  // descriptor, tile
};
struct BFin {
    const double *part;
    int count;
    double *scal;
    int ascale;  // 0: alpha = 1; 1 + j: alpha = 2^j ||r||_inf
};
enum { BK_SMOOTH2 = 0, BK_SMOOTH2_SCALED = 1, BK_SWEEP = 2, BK_PROLONG = 3, BK_OUTER = 4 };

hipError_t launch_batched_stencil(int kind, int V, int pf, int pc, const BDesc *d, const BItem *items, int nitems,
                                  const int *active, double omega, double *part, int grid, hipStream_t st);
hipError_t launch_batched_restrict(int V, int pf, int pc, const BDesc *d, const BItem *items, int nitems,
                                   const int *active, int grid, int threads, size_t lds, hipStream_t st);
hipError_t launch_batched_coarse(int prec, const BDesc *d, int n, const int *active, hipStream_t st);
// LDS-plane forms (grids of pitch >= 16; one pitch per launch, block size
// (ty + 2) P / V for the stencil kinds, (2 tyc + 3) P / V for the restriction).
hipError_t launch_batched_march(int kind, int V, int pf, int pc, const BDesc *d, const BItem *items, int nitems,
                                const int *active, double omega, double *part, int grid, int threads, size_t lds,
                                hipStream_t st);
hipError_t launch_batched_restrict2(int V, int pf, int pc, bool xsh, const BDesc *d, const BItem *items, int nitems,
                                    const int *active, int grid, int threads, size_t lds, hipStream_t st);
hipError_t launch_batched_finalize(const BFin *fin, int ninst, const int *active, hipStream_t st);

// ---- many right-hand sides, interleaved [z][y][x][k] -------------------------
// Arguments of one interleaved stage launch (unused members may stay null).
struct MArgs {
    int prec = 0;        // level storage format
    int pc = 0;          // coarse format (prolongation: of ec; restriction: of cout)
    int P = 0, K = 0;    // pitch of the level, number of right-hand sides
    int zc = 1;          // planes per thread (restriction: coarse planes)
    const void *b = nullptr;       // right-hand side (level format, or FP64 residual when aliased)
    const double *r = nullptr;     // scaled first smoothing: FP64 residual
    const double *inv = nullptr;   // 1/alpha_k (K values)
    const int *act = nullptr;      // per-column flags (K values)
    void *bout = nullptr;          // scaled first smoothing: round(r/alpha) out
    const void *cin = nullptr;     // input correction
    const void *ec = nullptr;      // coarse correction (prolongation)
    void *cout = nullptr;          // output correction, or coarse right-hand side (restriction)
    double omega = 0.8;
};
enum { MS_SMOOTH2 = 0, MS_SWEEP = 1 };

int m_vec(int prec);
bool m_supported(int prec, int K);
int m_stencil_blocks(int prec, int P, int K, int zc);
int m_update_blocks(int prec, int P, int K, int zc);  // workgroups (and partials) of the update
int m_resid_blocks(int n);
hipError_t launch_m_stage(int kind, const MArgs &a, hipStream_t st);
hipError_t launch_m_update(const MArgs &a, double *R, double *U, const double *alpha, double h2, double *part,
                           hipStream_t st);
hipError_t launch_m_coarse(int prec, int K, const void *b, void *c, hipStream_t st);
hipError_t launch_m_resid(int n, int P, int K, const double *b, const double *U, double *R, double *uout,
                          const int *mask, double inv_h2, double *part, hipStream_t st);
hipError_t launch_m_pack(int n, int P, int K, const double *src, double *dst, const int *keep, hipStream_t st);
hipError_t launch_m_finalize(const double *part, int nparts, int K, double *scal, const int *mask, int scaling,
                             hipStream_t st);
// Two-pass restriction: the fine residual (accumulator type, m_resid_bytes
// for a level of `elems` values) into rbuf, then full weighting into a.cout.
size_t m_resid_bytes(int prec, size_t elems);
hipError_t launch_m_restrict2(const MArgs &a, void *rbuf, int zcc, hipStream_t st);
// c = round(c + 4 P e) in place on a.cin (then a plain sweep completes the
// prolongation stage).
hipError_t launch_m_prolong_field(const MArgs &a, hipStream_t st);

// ---- the V-cycle on a caller-given scratch array (host side, mg_api.cpp) -----
// Bytes the V-cycle of a single-grid handle touches (its level vectors and
// base-level scratch; the leading part of the workspace layout).
mg_status_t vcycle_scratch_need(mg_handle h, size_t *bytes);
// mg_vcycle with ws (cap bytes, 256-byte aligned) in place of the bound
// workspace: clears the first vcycle_scratch_need bytes with a kernel, runs
// pack, V-cycle and unpack on stream; nothing is allocated.
mg_status_t vcycle_in(mg_handle h, void *ws, size_t cap, const void *b, void *c, void *stream);
// Set the thread's mg_last_error text and return s.
mg_status_t set_error(mg_status_t s, const char *msg);

}  // namespace mg
