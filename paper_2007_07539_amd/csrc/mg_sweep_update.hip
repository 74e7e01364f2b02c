// The last post-smoothing sweep of the finest level fused with the
// refinement update of Algorithm 2 (3-D):
//   c' = round_T(c + k (b - (6 c - nb(c))))          (damped Jacobi)
//   u += alpha h^2 c',  r -= alpha (6 c' - nb(c'))     (FP64)
// plus the (sum r^2, max |r|) partials of the block.  c' never goes to HBM:
// the kernel reads c, b, r, u and writes r, u (2 s + 32 bytes per point
// instead of 3 s for the sweep and s + 32 for the update).
//
// Two variants change what is read and written, not the arithmetic:
//   ALIAS  the right-hand side is formed from the residual r itself: b =
//          round_T(r / alpha), the value the first smoothing stored (for the
//          FP64 map without residual scaling, alpha = 1 and b is r).  A block
//          reads r on halo rows that its neighbours update, so the new
//          residual goes to a second array (Rout != R, swapped every step),
//          and r of a point is the row the block already holds: c, r and u
//          read, r and u written (s + 32 bytes per point instead of 2 s + 32).
//   DEFER  the update of u is postponed: c' is stored in its storage format
//          in slot k of a ring of corrections (k read from *ctr) and alpha in
//          adef[k]; launch_defer_flush later forms u += alpha_j h^2 c'_j for
//          the slots in order, the same roundings in the same sequence.  Per
//          step the kernel then reads c, b, r and writes r and c' (3 s + 16
//          bytes per point instead of 2 s + 32).
//
// A block owns TY output rows of full width and a chunk of planes.  The
// update at plane z needs c' on rows y0-1 .. y0+TY and planes z-1 .. z+1, so
// the sweep runs one plane ahead on TY + 2 rows, which needs c on TY + 4
// rows.  Thread row groups gi = 0 .. TY+3 hold fine rows y0-2+gi.  Per
// iteration w the sweep produces c' of plane w+1 and the update consumes
// plane w; c (plane w+1) and c' (plane w) sit in double-buffered LDS slots
// (rows chunk-major, LdsRun),
// one barrier per iteration: every LDS slot written in an iteration is written
// after its barrier and is not read again before the next one.  The arithmetic
// is that of the separate sweep and update kernels, operation for operation.
#include "mg_device.h"
#include "mg_launch.h"

#include <type_traits>

namespace mg {
namespace {

// FP64 rows need more registers than a 1024-thread block leaves a thread
template <class T> constexpr int su_bound() { return sizeof(T) == 8 ? 768 : 1024; }

template <int V, class T, bool ALIAS, bool DEFER>
__global__ __launch_bounds__(su_bound<T>()) void k_sweep_update(
    const T *__restrict__ c, const T *__restrict__ b, const double *R, double *Rout, double *__restrict__ U,
    T *__restrict__ Cd, const int *__restrict__ ctr, size_t cstride, double *__restrict__ adef,
    const double *__restrict__ scal, double h2, double omega, double *__restrict__ part, int P, int TY, int zc,
    int ytiles, int xcd) {
    typedef acc_t<T> A;
    typedef typename std::conditional<ALIAS, double, T>::type TB;  // what the b queue holds
    typedef LdsRun<T, V> LR;  // LDS rows, chunk-major
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[32];
    const int G = TY + 4;
    const size_t slot = (size_t)G * P;
    T *cs = reinterpret_cast<T *>(smem_raw);  // [2][G][P]: c of the plane being swept
    T *fs = cs + 2 * slot;                    // [2][G][P]: c' of the plane being updated
    const Grid<3> g{P};
    int blk = blockIdx.x;
    if (xcd) {
        const int nb = gridDim.x;
        blk = xcd_block(blk, nb);
    }
    const int yt = blk % ytiles, zch = blk / ytiles;
    const int y0 = 1 + yt * TY;
    const int z0 = 1 + zch * zc;
    const int z1 = min(z0 + zc, P);
    const int TXR = P / V;
    const int xc = threadIdx.x % TXR, gi = threadIdx.x / TXR;
    const int y = y0 - 2 + gi;
    const int x0 = xc * V;
    const bool row_in = y >= 1 && y <= P - 1;
    const bool sweep_row = gi >= 1 && gi <= TY + 2;
    const bool out_row = gi >= 2 && gi <= TY + 1 && y <= P - 1;
    const A k = (A)(omega / 6.0);
    const double a = scal[0];
    const double inv = scal[1];  // ALIAS: b = round_T(r * (1 / alpha)), as the first smoothing formed it
    const TB *bsrc = ALIAS ? reinterpret_cast<const TB *>(R) : reinterpret_cast<const TB *>(b);
    const double ah2 = a * h2;
    T *cd = nullptr;  // DEFER: this step's slot
    if constexpr (DEFER) {
        const int k = *ctr;
        cd = Cd + (size_t)k * cstride;
        if (blockIdx.x == 0 && threadIdx.x == 0) adef[k] = a;
    }

    auto fetch_c = [&](int z, RawRow<T, V> &r) {
        if (!row_in || z <= 0 || z >= P) {
            zero_row(r);
            return;
        }
        fetch_row<T, V>(c + g.at(x0, y, z), r);
    };
    // c of the own row: planes s-1, s, s+1 around the plane s being swept
    A pm[V], pc[V], pp[V];
    // c' of the own row: planes w-1, w, w+1 around the plane w being updated
    A fm[V], fc[V], fp[V];
    RawRow<T, V> cnext;       // c, plane s + 2
    RawRow<TB, V> bcur, bnext; // b (ALIAS: r), planes s and s + 1
    RawRow<double, V> rcur, ucur, rnext, unext;
    double ss = 0.0, mx = 0.0;
#pragma unroll
    for (int i = 0; i < V; ++i) fm[i] = fc[i] = A(0);

    const int wb = z0 - 2;  // first iteration: sweep plane z0 - 1
    {
        RawRow<T, V> t;
        fetch_c(wb, t);  // plane s - 1 of the first sweep
        widen_row<T, V>(t, pm);
        fetch_c(wb + 1, t);
        widen_row<T, V>(t, pc);
        T st[V];
#pragma unroll
        for (int i = 0; i < V; ++i) st[i] = Store<T>::from_acc(pc[i]);
        LR::store(cs + (size_t)((wb + 1) & 1) * slot + (size_t)gi * P, xc, TXR, st);
        fetch_c(wb + 2, t);
        widen_row<T, V>(t, pp);
        fetch_c(wb + 3, cnext);
        const int s0 = wb + 1;
        if (sweep_row && row_in && s0 >= 1 && s0 <= P - 1) fetch_row<TB, V>(bsrc + g.at(x0, y, s0), bnext);
        if (out_row && z0 < z1) {
            if constexpr (!ALIAS) fetch_row<double, V>(R + g.at(x0, y, z0), rnext);
            if constexpr (!DEFER) fetch_row<double, V>(U + g.at(x0, y, z0), unext);
        }
    }
    for (int w = wb; w < z1; ++w) {
        const int s = w + 1;  // plane swept in this iteration
        if constexpr (ALIAS) {
            if (w >= z0) rcur = bcur;  // b of plane w is its residual
        }
        bcur = bnext;
        if (sweep_row && row_in && s + 1 >= 1 && s + 1 <= P - 1 && s + 1 <= z1)
            fetch_row<TB, V>(bsrc + g.at(x0, y, s + 1), bnext);
        if (w >= z0) {
            if constexpr (!ALIAS) rcur = rnext;
            if constexpr (!DEFER) ucur = unext;
            if (out_row && w + 1 < z1) {
                if constexpr (!ALIAS) fetch_row<double, V>(R + g.at(x0, y, w + 1), rnext);
                if constexpr (!DEFER) fetch_row<double, V>(U + g.at(x0, y, w + 1), unext);
            }
        }
        __syncthreads();
        // sweep of plane s on rows gi = 1 .. TY+2
        if (sweep_row) {
            T o[V];
            if (row_in && s >= 1 && s <= P - 1) {
                const T *row = cs + (size_t)(s & 1) * slot + (size_t)gi * P;
                A nb[V];
                const A xl = x0 > 0 ? (A)widen(LR::left_of(row, xc, TXR)) : A(0);
                const A xr = x0 + V < P ? (A)widen(LR::right_of(row, xc, TXR)) : A(0);
#pragma unroll
                for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? pc[i - 1] : xl) + (i < V - 1 ? pc[i + 1] : xr);
                A ym[V], yp[V], bv[V];
                LR::load(row - P, xc, TXR, ym);
                LR::load(row + P, xc, TXR, yp);
                if constexpr (ALIAS) {
                    double rv[V];
                    widen_row<double, V>(bcur, rv);
#pragma unroll
                    for (int i = 0; i < V; ++i) bv[i] = (A)widen(Store<T>::from_f64(rv[i] * inv));
                } else {
                    widen_row<T, V>(bcur, bv);
                }
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    nb[i] += ym[i];
                    nb[i] += yp[i];
                    nb[i] += pm[i];
                    nb[i] += pp[i];
                    const A lc = fmaT<A>(A(6), pc[i], -nb[i]);
                    o[i] = Store<T>::from_acc(fmaT<A>(k, bv[i] - lc, pc[i]));
                }
                if (x0 == 0) o[0] = zero_of<T>();
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) o[i] = zero_of<T>();
            }
#pragma unroll
            for (int i = 0; i < V; ++i) fp[i] = (A)widen(o[i]);
            LR::store(fs + (size_t)(s & 1) * slot + (size_t)gi * P, xc, TXR, o);
        }
        // update of plane w = s - 1 on rows gi = 2 .. TY+1, c' of plane w in LDS
        if (w >= z0 && out_row) {
            const T *row = fs + (size_t)(w & 1) * slot + (size_t)gi * P;
            double cv[V], nb[V];
#pragma unroll
            for (int i = 0; i < V; ++i) cv[i] = (double)fc[i];
            const double xl = x0 > 0 ? (double)widen(LR::left_of(row, xc, TXR)) : 0.0;
            const double xr = x0 + V < P ? (double)widen(LR::right_of(row, xc, TXR)) : 0.0;
#pragma unroll
            for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? cv[i - 1] : xl) + (i < V - 1 ? cv[i + 1] : xr);
            double ym[V], yp[V];
            LR::load(row - P, xc, TXR, ym);
            LR::load(row + P, xc, TXR, yp);
            double r[V], u[V];
            widen_row<double, V>(rcur, r);
            if constexpr (!DEFER) widen_row<double, V>(ucur, u);
#pragma unroll
            for (int i = 0; i < V; ++i) {
                nb[i] += ym[i];
                nb[i] += yp[i];
                nb[i] += (double)fm[i];
                nb[i] += (double)fp[i];
                const double lc = fmaT<double>(6.0, cv[i], -nb[i]);
                r[i] = fmaT<double>(-a, lc, r[i]);
                if constexpr (!DEFER) u[i] = fmaT<double>(ah2, cv[i], u[i]);
            }
            if (x0 == 0) r[0] = 0.0, u[0] = 0.0;
#pragma unroll
            for (int i = 0; i < V; ++i) {
                ss += r[i] * r[i];
                mx = nanmax(mx, fabs(r[i]));
            }
            const size_t at = g.at(x0, y, w);
            store_row<double, V>(Rout + at, r);
            if constexpr (DEFER) {
                // c' is a value of T (rounded by the sweep), so this is exact
                T co[V];
#pragma unroll
                for (int i = 0; i < V; ++i) co[i] = Store<T>::from_acc(fc[i]);
                store_row<T, V>(cd + at, co);
            } else {
                store_row<double, V>(U + at, u);
            }
        }
        // c of plane s + 1 for the next iteration's y neighbours (that slot was
        // last read before this iteration's barrier)
        {
            T st[V];
#pragma unroll
            for (int i = 0; i < V; ++i) st[i] = Store<T>::from_acc(pp[i]);
            LR::store(cs + (size_t)((s + 1) & 1) * slot + (size_t)gi * P, xc, TXR, st);
        }
        // advance the queues
#pragma unroll
        for (int i = 0; i < V; ++i) {
            pm[i] = pc[i];
            pc[i] = pp[i];
            fm[i] = fc[i];
            fc[i] = fp[i];
        }
        widen_row<T, V>(cnext, pp);
        fetch_c(s + 3, cnext);
    }
    block_reduce(ss, mx, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss;
        part[2 * blockIdx.x + 1] = mx;
    }
}

template <class T, bool ALIAS, bool DEFER>
hipError_t sweep_update_t(int P, const SweepUpdateArgs &q, const Shape &s, hipStream_t st) {
    const int ytiles = (P - 1 + s.ty - 1) / s.ty;
    const int nch = (P - 1 + s.zc - 1) / s.zc;
    const int threads = (P / s.V) * (s.ty + 4);
    const size_t lds = sweep_update_lds_bytes(P, s.ty, sizeof(T));
    hipLaunchKernelGGL((k_sweep_update<4, T, ALIAS, DEFER>), dim3(ytiles * nch), dim3(threads), lds, st,
                       static_cast<const T *>(q.c), static_cast<const T *>(q.b), q.R, q.Rout, q.U,
                       static_cast<T *>(q.cdefer), q.ctr, q.cstride, q.adef, q.scal, q.h2, q.omega, q.part, P, s.ty,
                       s.zc, ytiles, s.xcd);
    return hipGetLastError();
}

template <class T> hipError_t sweep_update_mode(int P, const SweepUpdateArgs &q, const Shape &s, hipStream_t st) {
    const bool alias = q.b == (const void *)q.R, defer = q.cdefer != nullptr;
    if (alias) {
        if (q.Rout == q.R) return hipErrorInvalidValue;  // the residual must not be updated in place
        return defer ? sweep_update_t<T, true, true>(P, q, s, st) : sweep_update_t<T, true, false>(P, q, s, st);
    }
    return defer ? sweep_update_t<T, false, true>(P, q, s, st) : sweep_update_t<T, false, false>(P, q, s, st);
}

}  // namespace

size_t sweep_update_lds_bytes(int P, int ty, size_t sb) { return 4 * (size_t)(ty + 4) * P * sb; }

// the kernel's own 256 bytes of reduction scratch come out of the same LDS
constexpr size_t kSuDynLdsMax = kLdsMax - 1024;

hipError_t sweep_update_prepare() {
    static hipError_t done = [] {
        const void *fns[] = {
#define MG_SU_FN(T)                                                                                       \
    (const void *)k_sweep_update<4, T, false, false>, (const void *)k_sweep_update<4, T, false, true>,       \
        (const void *)k_sweep_update<4, T, true, false>, (const void *)k_sweep_update<4, T, true, true>
            MG_SU_FN(double), MG_SU_FN(float), MG_SU_FN(f16), MG_SU_FN(bf16)
#undef MG_SU_FN
        };
        for (const void *f : fns) {
            // what the function's static LDS leaves of the workgroup's kLdsMax
            hipFuncAttributes fa{};
            hipError_t e = hipFuncGetAttributes(&fa, f);
            if (e == hipSuccess && fa.sharedSizeBytes + kSuDynLdsMax > kLdsMax) e = hipErrorInvalidValue;
            if (e == hipSuccess)
                e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)(kLdsMax - fa.sharedSizeBytes));
            if (e != hipSuccess) {
                (void)hipGetLastError();  // leave no error for the next launch to report
                return e;
            }
        }
        return hipSuccess;
    }();
    return done;
}

bool sweep_update_ok(int P, int prec, const Shape &s) {
    // V = 4 only: at V = 8 the FP64 rows of the update spill registers
    if (s.V != 4 || s.V > P || s.ty < 1 || s.ty > P - 1 || s.zc < 1 || s.zc > P - 1) return false;
    if ((P / s.V) * (s.ty + 4) > (prec == P_F64 ? 768 : 1024)) return false;
    return sweep_update_lds_bytes(P, s.ty, prec_bytes(prec)) <= kSuDynLdsMax;
}

int sweep_update_blocks(int P, const Shape &s) { return ((P - 1 + s.ty - 1) / s.ty) * ((P - 1 + s.zc - 1) / s.zc); }

hipError_t launch_sweep_update(int prec, int P, const SweepUpdateArgs &q, const Shape &s, hipStream_t st) {
    if (!sweep_update_ok(P, prec, s)) return hipErrorInvalidValue;
    if (sweep_update_lds_bytes(P, s.ty, prec_bytes(prec)) > 65536 && sweep_update_prepare() != hipSuccess)
        return hipErrorInvalidValue;
    switch (prec) {
    case P_F64: return sweep_update_mode<double>(P, q, s, st);
    case P_F32: return sweep_update_mode<float>(P, q, s, st);
    case P_F16: return sweep_update_mode<f16>(P, q, s, st);
    case P_BF16: return sweep_update_mode<bf16>(P, q, s, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace mg
