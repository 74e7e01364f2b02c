// A level's first pre-smoothing (two sweeps from zero) fused with the residual
// and full-weighting restriction of its result (3-D).  On the finest level
// inside a refinement step the right-hand side is the scaled residual:
//   b  = round_T(r / alpha)                     (residuum scaling and cast)
//   c1 = round_T(k b),  c2 = round_T(c1 + k (b - (6 c1 - nb(c1))))
//   b_c = round_TC(FW(b - (6 c2 - nb(c2))))
// b and c2 are written for the later sweeps and the prolongation; c2 is
// restricted from registers and LDS instead of being read back from HBM
// (8 + 2 s + s_c/8 bytes per point instead of 8 + 2 s, then 2 s + s_c/8).  On
// a coarser level b is the stored right-hand side and only c2 and b_c are
// written (2 s + s_c/8 instead of 2 s, then 2 s + s_c/8).
//
// A block owns tyc coarse rows and zcc coarse planes, like the pipelined
// restriction kernel.  Its thread row groups gi = 0 .. 2 tyc + 4 hold fine
// rows 2 Y0 - 3 + gi: the residual rows 2 Y0 - 1 .. 2 Y0 + 2 tyc - 1 need c2
// one row further out, which needs c1 one more row out.  Per iteration t the
// block forms c2 of plane t+1 (from c1 of planes t .. t+2), the residual of
// plane t (from c2 of planes t-1 .. t+1), and folds the residual rows of
// plane t-1 into the coarse plane; c1, c2 and the residual rows sit in
// double-buffered LDS slots (in the accumulator format: FP32, up to 104 KB at
// P = 512, or FP64 for an FP64 level, 124 KB at P = 512 with one coarse row
// per tile; gfx950 allows one workgroup 160 KB), each written after the
// iteration's barrier and not read again before the next one.  LDS rows are
// stored chunk-major (LdsRun) so that the wave's 16-byte accesses do not
// conflict.  The arithmetic is that of the
// separate kernels, operation for operation, so results are bitwise equal.
#include "mg_device.h"
#include "mg_launch.h"

#include <type_traits>

namespace mg {
namespace {

template <class T> constexpr int prec_of_t() {
    return sizeof(T) == 8 ? P_F64 : sizeof(T) == 4 ? P_F32 : std::is_same<T, f16>::value ? P_F16 : P_BF16;
}

// SCALED: the right-hand side is the scaled-and-cast FP64 residual (the
// finest level inside a refinement step; b is also written out); otherwise
// it is the level's stored b (a coarser level, or a V-cycle on its own).
// FP64 levels: four values per thread (two waves per fine row of P = 512, twice
// the waves of eight per thread); the fine residual rows then go to LDS as
// they are and the coarse threads apply the x weights (XW), since a row's
// left neighbour value may sit in the other wave.  Same operations, same order.
template <class T> constexpr int sr_vec() { return sizeof(T) == 8 ? 4 : 8; }
template <class T> constexpr int sr_bound() { return sizeof(T) == 8 ? 1024 : 768; }

// NARROW: c1 and c2 sit in LDS in the storage format T instead of the
// accumulator format (exact: both are values of T), which halves that part of
// the LDS so that two workgroups fit a CU; they are widened when read.
template <class T, class TC, bool SCALED, bool NARROW>
__global__ __launch_bounds__(sr_bound<T>()) void k_smooth_restrict(const void *__restrict__ src,
                                                          const double *__restrict__ scal, T *__restrict__ bout,
                                                          T *__restrict__ cout, TC *__restrict__ bc, int P, int tyc,
                                                          int zcc, int ytiles, double omega, int xcd) {
    constexpr int V = sr_vec<T>(), VC = V / 2;
    constexpr bool XW = V == 4;  // x weights in the coarse threads, from raw residual rows
    typedef acc_t<T> A;
    typedef typename std::conditional<NARROW, T, A>::type LC;  // LDS format of c1 and c2
    typedef LdsRun<LC, V> LR;   // fine rows in LDS, chunk-major
    typedef LdsRun<A, XW ? V : VC> LRC;  // residual rows: raw (XW) or x-weighted
    typedef typename std::conditional<SCALED, double, T>::type S;  // source format
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int G = 2 * tyc + 5, RR = 2 * tyc + 1, RW = XW ? P : P / 2;
    const size_t cslot = (size_t)G * P, rslot = (size_t)RR * RW;
    // c1 and c2 sit in LDS widened to the accumulator type, so that neither
    // their stores nor their loads convert
    LC *c1s = reinterpret_cast<LC *>(smem_raw);  // [2][G][P]
    LC *c2s = c1s + 2 * cslot;                   // [2][G][P]
    A *rs = reinterpret_cast<A *>(c2s + 2 * cslot);  // [2][RR][RW]
    const int Pc = P >> 1, TXR = P / V;
    const Grid<3> gc{Pc};
    int blk = blockIdx.x;
    if (xcd) {
        const int nb = gridDim.x;
        blk = xcd_block(blk, nb);
    }
    const int ytile = blk % ytiles, zch = blk / ytiles;
    const int Y0 = 1 + ytile * tyc;
    const int Z0 = 1 + zch * zcc, Z1 = min(Z0 + zcc, Pc);
    const int zf0 = 2 * Z0 - 1, zf1 = 2 * Z1 - 1;
    const int xc = threadIdx.x % TXR, gi = threadIdx.x / TXR;
    const int y = 2 * Y0 - 3 + gi;
    const int x0 = xc * V, X0 = xc * VC;
    const bool row_in = y >= 1 && y <= P - 1;
    const bool c2_row = gi >= 1 && gi <= G - 2;
    const bool res_slot = gi >= 2 && gi <= G - 3;
    const bool res_row = res_slot && row_in;
    // fine rows 2 Y0 - 1 .. 2 Y0 + 2 tyc - 2 belong to this tile; the last
    // tile also owns the last fine row P - 1
    const bool own_row = row_in && y >= 2 * Y0 - 1 && (y <= 2 * Y0 + 2 * tyc - 2 || Y0 + tyc >= Pc);
    const bool last_z = Z1 == Pc;
    auto own_plane = [&](int z) { return z >= zf0 && (z <= zf1 - 1 || (last_z && z == P - 1)); };
    const bool coarse = gi < tyc && Y0 + gi < Pc;
    const int Yc = Y0 + gi;
    const double inv = SCALED ? scal[1] : 1.0;
    const A k = (A)(omega / 6.0);
    // offsets of the own row (plane 0) and of plane z, the latter uniform
    const size_t roff = (size_t)(long)y * P + x0;
    const size_t PP = (size_t)P * P;
    auto at = [&](int z) { return (size_t)z * PP + roff; };

    auto fetch_r = [&](int z, RawRow<S, V> &rr) {
        if (!row_in || z < 1 || z > P - 1) {
            zero_row(rr);
            return;
        }
        fetch_row<S, V>(static_cast<const S *>(src) + at(z), rr);
    };
    // b of the own row (zero outside the interior), as stored (braw) and
    // widened (bw): round_T(r / alpha), or the stored b itself
    auto scaled = [&](const RawRow<S, V> &rr, T (&braw)[V], A (&bw)[V]) {
        if constexpr (SCALED) {
            double rv[V];
            widen_row<double, V>(rr, rv);
#pragma unroll
            for (int i = 0; i < V; ++i) {
                braw[i] = Store<T>::from_f64(rv[i] * inv);
                bw[i] = widen(braw[i]);
            }
        } else {
            widen_row<T, V>(rr, bw);
        }
    };
    // c1 = round_T(k b), widened
    auto first = [&](const A (&bw)[V], A (&kw)[V]) {
#pragma unroll
        for (int i = 0; i < V; ++i) kw[i] = round_to<T>(k * bw[i]);
    };

    // Per plane the block keeps b, c1 and c2 of the own row in registers,
    // three planes each; the loop body is written out three times with the
    // roles of the arrays rotated, so that no values are moved between planes.
    A bA[V], bB[V], bC[V];   // b
    A kA[V], kB[V], kC[V];   // c1
    A cA[V], cB[V], cC[V];   // c2
    RawRow<S, V> rnext;      // source row of the own row, plane t+2 (then t+3)
    A acc[VC];
#pragma unroll
    for (int j = 0; j < VC; ++j) acc[j] = A(0);
#pragma unroll
    for (int i = 0; i < V; ++i) cA[i] = cB[i] = cC[i] = A(0);

    const int tb = zf0 - 2;
    {
        RawRow<S, V> t0;
        T braw[V];
        fetch_r(tb, t0);
        scaled(t0, braw, bA);
        first(bA, kA);
        fetch_r(tb + 1, t0);
        scaled(t0, braw, bB);
        first(bB, kB);
        LR::store(c1s + (size_t)((tb + 1) & 1) * cslot + (size_t)gi * P, xc, TXR, kB);
        fetch_r(tb + 2, rnext);
    }

    // fold the x-weighted residual rows of fine plane zf (slot s) into acc
    auto coarse_step = [&](int zf, int s) {
        const A *rb = rs + (size_t)s * rslot;
        const int j = zf - zf0;
        const bool last_of_z = j > 0 && (j & 1) == 0;  // zf = 2Z + 1
        A xs[3][VC];
        if constexpr (XW) {
            // fine residuals x0 - 1 .. x0 + 3 of each of the three rows, then
            // the x weights exactly as a fine thread forms them
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                const A *row = rb + (size_t)(2 * gi + oy) * RW;
                A r[V];
                LRC::load(row, xc, TXR, r);
                const A left = xc > 0 ? LRC::left_of(row, xc, TXR) : A(0);
#pragma unroll
                for (int jj = 0; jj < VC; ++jj) {
                    const A lm = jj > 0 ? r[2 * jj - 1] : left;
                    xs[oy][jj] = A(0.25) * (lm + r[2 * jj + 1]) + A(0.5) * r[2 * jj];
                }
                if (xc == 0) xs[oy][0] = A(0);
            }
        } else {
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) LRC::load(rb + (size_t)(2 * gi + oy) * RW, xc, TXR, xs[oy]);
        }
        TC out[VC];
#pragma unroll
        for (int jx = 0; jx < VC; ++jx) {
            const int X = X0 + jx;
            A q = A(0);
            if (X >= 1) q = A(0.25) * (xs[0][jx] + xs[2][jx]) + A(0.5) * xs[1][jx];
            if (j == 0) {
                acc[jx] = A(0.25) * q;
            } else if (!last_of_z) {
                acc[jx] += A(0.5) * q;
            } else {
                out[jx] = store_as<TC>(acc[jx] + A(0.25) * q);
                acc[jx] = A(0.25) * q;
            }
        }
        if (last_of_z) {
            if (X0 == 0) out[0] = store_as<TC>(A(0));
            store_row<TC, VC>(bc + gc.at(X0, Yc, (zf - 1) >> 1), out);
        }
    };

    // One plane step: b0, b1 = b of planes t, t+1 and b2 <- b of plane t+2;
    // k0, k1 = c1 of t, t+1 and k2 <- c1 of t+2; c0, c1 = c2 of t-1, t and
    // c2 <- c2 of t+1.
    auto body = [&](int t, const A (&b0)[V], const A (&b1)[V], A (&b2)[V], const A (&k0)[V], const A (&k1)[V],
                    A (&k2)[V], const A (&c0)[V], const A (&c1)[V], A (&c2)[V]) __attribute__((always_inline)) {
        // b and c1 of plane t+2 (registers only before the barrier)
        T braw[V];
        scaled(rnext, braw, b2);
        fetch_r(t + 3, rnext);
        first(b2, k2);
        if constexpr (SCALED) {
            if (own_row && own_plane(t + 2)) {
                if (x0 == 0) braw[0] = zero_of<T>();
                store_row<T, V>(bout + at(t + 2), braw);
            }
        }
        __syncthreads();
        if (coarse && t - 1 >= zf0) coarse_step(t - 1, (t - 1) & 1);
        // c2 of plane t+1 on rows gi = 1 .. G-2
        if (c2_row) {
            const int p = t + 1;
            T craw[V];
            if (row_in && p >= 1 && p <= P - 1) {
                const LC *row = c1s + (size_t)(p & 1) * cslot + (size_t)gi * P;
                A nb[V];
                const A xl = x0 > 0 ? (A)widen(LR::left_of(row, xc, TXR)) : A(0);
                const A xr = x0 + V < P ? (A)widen(LR::right_of(row, xc, TXR)) : A(0);
#pragma unroll
                for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? k1[i - 1] : xl) + (i < V - 1 ? k1[i + 1] : xr);
                A ym[V], yp[V];
                LR::load(row - P, xc, TXR, ym);
                LR::load(row + P, xc, TXR, yp);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    nb[i] += ym[i];
                    nb[i] += yp[i];
                    nb[i] += k0[i];
                    nb[i] += k2[i];
                    const A lc = fmaT<A>(A(6), k1[i], -nb[i]);
                    craw[i] = Store<T>::from_acc(fmaT<A>(k, b1[i] - lc, k1[i]));
                    c2[i] = widen(craw[i]);
                }
                if (x0 == 0) craw[0] = zero_of<T>(), c2[0] = A(0);
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) craw[i] = zero_of<T>(), c2[i] = A(0);
            }
            LR::store(c2s + (size_t)(p & 1) * cslot + (size_t)gi * P, xc, TXR, c2);
            if (own_row && own_plane(p)) store_row<T, V>(cout + at(p), craw);
        }
        // residual of plane t on rows gi = 2 .. G-3, x weights in the thread
        if (t >= zf0) {
            A r[V];
            if (res_row) {
                const LC *row = c2s + (size_t)(t & 1) * cslot + (size_t)gi * P;
                A nb[V];
                const A xl = x0 > 0 ? (A)widen(LR::left_of(row, xc, TXR)) : A(0);
                const A xr = x0 + V < P ? (A)widen(LR::right_of(row, xc, TXR)) : A(0);
#pragma unroll
                for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? c1[i - 1] : xl) + (i < V - 1 ? c1[i + 1] : xr);
                A ym[V], yp[V];
                LR::load(row - P, xc, TXR, ym);
                LR::load(row + P, xc, TXR, yp);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    nb[i] += ym[i];
                    nb[i] += yp[i];
                    nb[i] += c0[i];
                    nb[i] += c2[i];
                    r[i] = b0[i] - fmaT<A>(A(6), c1[i], -nb[i]);
                }
                if (x0 == 0) r[0] = A(0);
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) r[i] = A(0);
            }
            if constexpr (XW) {
                // the raw residual row; the coarse threads weight it
                if (res_slot) LRC::store(rs + (size_t)(t & 1) * rslot + (size_t)(gi - 2) * RW, xc, TXR, r);
            } else {
                // coarse X = x0/2 + j takes fine 2X-1, 2X, 2X+1; x0-1 from the previous lane
                const A left_in = __shfl_up(r[V - 1], 1, 64);
                const A left = x0 > 0 ? left_in : A(0);
                A xq[VC];
#pragma unroll
                for (int j = 0; j < VC; ++j) {
                    const A lm = j > 0 ? r[2 * j - 1] : left;
                    xq[j] = A(0.25) * (lm + r[2 * j + 1]) + A(0.5) * r[2 * j];
                }
                if (x0 == 0) xq[0] = A(0);
                if (res_slot) LRC::store(rs + (size_t)(t & 1) * rslot + (size_t)(gi - 2) * RW, xc, TXR, xq);
            }
        }
        // c1 of plane t+2 for the next step's neighbours
        LR::store(c1s + (size_t)((t + 2) & 1) * cslot + (size_t)gi * P, xc, TXR, k2);
    };

    for (int t = tb;;) {
        body(t, bA, bB, bC, kA, kB, kC, cA, cB, cC);
        if (++t > zf1) break;
        body(t, bB, bC, bA, kB, kC, kA, cB, cC, cA);
        if (++t > zf1) break;
        body(t, bC, bA, bB, kC, kA, kB, cC, cA, cB);
        if (++t > zf1) break;
    }
    __syncthreads();
    if (coarse) coarse_step(zf1, zf1 & 1);
}

template <class T, bool SCALED, bool NARROW>
hipError_t smooth_restrict_t(int pc, int P, const void *src, const double *scal, void *bout, void *cout, void *bc,
                             double omega, const RShape &s, hipStream_t st) {
    const int Pc = P / 2;
    const int ytiles = (Pc - 1 + s.tyc - 1) / s.tyc;
    const int blocks = ytiles * ((Pc - 1 + s.zcc - 1) / s.zcc);
    const int threads = (2 * s.tyc + 5) * (P / sr_vec<T>());
    const size_t lds = smooth_restrict_lds_bytes(P, s.tyc, prec_of_t<T>(), NARROW);
#define MG_SR(TCT)                                                                                                     \
    hipLaunchKernelGGL((k_smooth_restrict<T, TCT, SCALED, NARROW>), dim3(blocks), dim3(threads), lds, st, src,     \
                       scal, static_cast<T *>(bout), static_cast<T *>(cout), static_cast<TCT *>(bc), P, s.tyc,     \
                       s.zcc, ytiles, omega, 1)
    switch (pc) {
    case P_F64: MG_SR(double); break;
    case P_F32: MG_SR(float); break;
    case P_F16: MG_SR(f16); break;
    case P_BF16: MG_SR(bf16); break;
    default: return hipErrorInvalidValue;
    }
#undef MG_SR
    return hipGetLastError();
}

}  // namespace

size_t smooth_restrict_lds_bytes(int P, int tyc, int prec, bool narrow) {
    const size_t acc = prec == P_F64 ? sizeof(double) : sizeof(float);
    const size_t lc = narrow ? prec_bytes(prec) : acc;
    const size_t rw = prec == P_F64 ? P : P / 2;  // raw residual rows for FP64 (XW)
    return 4 * (size_t)(2 * tyc + 5) * P * lc + 2 * (size_t)(2 * tyc + 1) * rw * acc;
}

hipError_t smooth_restrict_prepare() {
    static hipError_t done = [] {
        const void *fns[] = {
#define MG_SR_FN(T, S, N)                                                                                     \
    (const void *)k_smooth_restrict<T, double, S, N>, (const void *)k_smooth_restrict<T, float, S, N>,        \
        (const void *)k_smooth_restrict<T, f16, S, N>, (const void *)k_smooth_restrict<T, bf16, S, N>
            MG_SR_FN(double, true, false), MG_SR_FN(float, true, false), MG_SR_FN(f16, true, false),
            MG_SR_FN(bf16, true, false), MG_SR_FN(double, false, false), MG_SR_FN(float, false, false),
            MG_SR_FN(f16, false, false), MG_SR_FN(bf16, false, false), MG_SR_FN(f16, true, true),
            MG_SR_FN(bf16, true, true), MG_SR_FN(f16, false, true), MG_SR_FN(bf16, false, true)
#undef MG_SR_FN
        };
        for (const void *f : fns) {
            const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
            if (e != hipSuccess) {
                (void)hipGetLastError();  // leave no error for the next launch to report
                return e;
            }
        }
        return hipSuccess;
    }();
    return done;
}

bool smooth_restrict_ok(int P, int prec, const RShape &s) {
    // FP32/FP16/BF16: rows of P/8 threads within one wave (the x weights use a
    // lane shuffle); FP64: P/4 threads per row, no shuffle
    if (P < 16 || (prec != P_F64 && (P / 8 > 64 || 64 % (P / 8) != 0))) return false;
    if (s.tyc < 1 || s.tyc > P / 2 - 1 || s.zcc < 1 || s.zcc > P / 2 - 1) return false;
    // pipe 3: c1, c2 in LDS in FP32/FP64; 4: in the 2-byte storage format
    if (s.pipe != 3 && !(s.pipe == 4 && prec_bytes(prec) == 2)) return false;
    const int threads = (2 * s.tyc + 5) * (P / (prec == P_F64 ? 4 : 8));
    if (threads > (prec == P_F64 ? 1024 : 768)) return false;  // the kernel's launch bound
    return smooth_restrict_lds_bytes(P, s.tyc, prec, s.pipe == 4) <= kLdsMax;
}

hipError_t launch_smooth_restrict(int prec, int pc, int P, const double *R, const double *scal, void *bout,
                                  void *cout, void *bc, double omega, const RShape &s, hipStream_t st) {
    if (!smooth_restrict_ok(P, prec, s)) return hipErrorInvalidValue;
    const bool nw = s.pipe == 4;
    switch (prec) {
    case P_F64: return smooth_restrict_t<double, true, false>(pc, P, R, scal, bout, cout, bc, omega, s, st);
    case P_F32: return smooth_restrict_t<float, true, false>(pc, P, R, scal, bout, cout, bc, omega, s, st);
    case P_F16:
        return nw ? smooth_restrict_t<f16, true, true>(pc, P, R, scal, bout, cout, bc, omega, s, st)
                  : smooth_restrict_t<f16, true, false>(pc, P, R, scal, bout, cout, bc, omega, s, st);
    case P_BF16:
        return nw ? smooth_restrict_t<bf16, true, true>(pc, P, R, scal, bout, cout, bc, omega, s, st)
                  : smooth_restrict_t<bf16, true, false>(pc, P, R, scal, bout, cout, bc, omega, s, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_smooth_restrict_b(int prec, int pc, int P, const void *b, void *cout, void *bc, double omega,
                                    const RShape &s, hipStream_t st) {
    if (!smooth_restrict_ok(P, prec, s)) return hipErrorInvalidValue;
    const bool nw = s.pipe == 4;
    switch (prec) {
    case P_F64: return smooth_restrict_t<double, false, false>(pc, P, b, nullptr, nullptr, cout, bc, omega, s, st);
    case P_F32: return smooth_restrict_t<float, false, false>(pc, P, b, nullptr, nullptr, cout, bc, omega, s, st);
    case P_F16:
        return nw ? smooth_restrict_t<f16, false, true>(pc, P, b, nullptr, nullptr, cout, bc, omega, s, st)
                  : smooth_restrict_t<f16, false, false>(pc, P, b, nullptr, nullptr, cout, bc, omega, s, st);
    case P_BF16:
        return nw ? smooth_restrict_t<bf16, false, true>(pc, P, b, nullptr, nullptr, cout, bc, omega, s, st)
                  : smooth_restrict_t<bf16, false, false>(pc, P, b, nullptr, nullptr, cout, bc, omega, s, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace mg
