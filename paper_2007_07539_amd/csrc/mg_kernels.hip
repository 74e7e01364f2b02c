// gfx950 kernels of the mixed-precision multigrid V-cycle and the FP64
// iterative-refinement loop (Oo & Vogel, arXiv 2007.07539: Algorithm 1 for the
// cycle, Algorithm 2 for the refinement, Section 6 for the per-level formats).
//
// All level operators are matrix-free.  Corrections are kept in grid-scaled
// units c = e / h^2, so that on every level the operator is the integer
// stencil L = [2D on the centre, -1 on each face neighbour]; damped Jacobi is
// c' = c + k (b - L c) with k = omega / (2D); prolongation gains the factor
// (h_coarse / h_fine)^2 = 4.  Powers of two only, so the change of units is
// exact in every binary format.
//
// Work decomposition (all stencil kernels): a thread owns V consecutive x
// values of one row and marches along z, keeping the z-1, z, z+1 values of its
// own row in registers; the y and x neighbours come from the cache hierarchy
// (the same rows are the centre rows of neighbouring threads).  The
// residual+restriction kernel stages fine residual rows in LDS.
#include "mg_device.h"
#include "mg_launch.h"

#include <algorithm>
#include <type_traits>

namespace mg {

// ===========================================================================
// Field policies: the value of a grid function at a position, in accumulator
// type `acc`, already rounded to the format it would be stored in.  Positions
// on the boundary evaluate to zero.
// ===========================================================================

// A stored array.
template <class T, class A> struct FArr {
    typedef A acc;
    const T *__restrict__ p;
    template <int D, int V> __device__ __forceinline__ void row(const Grid<D> &g, int x0, int y, int z, A (&o)[V]) const {
        if (g.ghost_row(y, z)) {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = A(0);
            return;
        }
        load_row<T, V>(p + g.at(x0, y, z), o);  // x = 0 is a stored zero ghost
    }
    template <int D> __device__ __forceinline__ A one(const Grid<D> &g, int x, int y, int z) const {
        if (x <= 0 || x >= g.P || g.ghost_row(y, z)) return A(0);
        return (A)widen(p[g.at(x, y, z)]);
    }
};

// Right-hand side of the finest level inside the refinement loop:
// round_T(r * (1/alpha)) from the FP64 residual (the residuum scaling and
// precision change of Algorithm 2).
template <class T> struct FScaled {
    typedef acc_t<T> acc;
    const double *__restrict__ r;
    const double *__restrict__ scal;  // scal[1] = 1/alpha
    template <int D, int V> __device__ __forceinline__ void row(const Grid<D> &g, int x0, int y, int z, acc (&o)[V]) const {
        if (g.ghost_row(y, z)) {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = acc(0);
            return;
        }
        double rv[V];
        load_row<double, V>(r + g.at(x0, y, z), rv);
        const double inv = scal[1];
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = widen(Store<T>::from_f64(rv[i] * inv));
    }
    template <int D> __device__ __forceinline__ acc one(const Grid<D> &g, int x, int y, int z) const {
        if (x <= 0 || x >= g.P || g.ghost_row(y, z)) return acc(0);
        return widen(Store<T>::from_f64(r[g.at(x, y, z)] * scal[1]));
    }
};

// First Jacobi iterate from c = 0: round_T(k * b).
template <class T, class R> struct FJac0 {
    typedef acc_t<T> acc;
    R rhs;
    acc k;
    template <int D, int V> __device__ __forceinline__ void row(const Grid<D> &g, int x0, int y, int z, acc (&o)[V]) const {
        rhs.template row<D, V>(g, x0, y, z, o);
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = round_to<T>(k * o[i]);
    }
    template <int D> __device__ __forceinline__ acc one(const Grid<D> &g, int x, int y, int z) const {
        return round_to<T>(k * rhs.one(g, x, y, z));
    }
};

// Corrected fine correction round_TF(c + 4 P e_c): linear interpolation of
// the coarse correction (fine coordinate q sits on coarse q/2 when even,
// between (q-1)/2 and (q+1)/2 when odd).  Interpolation runs in FP64 when
// either level is FP64, else in FP32.
template <class TF, class TC> struct FProl {
    typedef acc_t<TF> acc;
    typedef typename std::conditional<std::is_same<TC, double>::value || std::is_same<TF, double>::value,
                                      double, float>::type PA;
    const TF *__restrict__ c;
    const TC *__restrict__ ec;
    int Pc;

    __device__ __forceinline__ static int split(int q, int (&Q)[2]) {
        if ((q & 1) == 0) {
            Q[0] = q >> 1;
            return 1;
        }
        Q[0] = (q - 1) >> 1;
        Q[1] = (q + 1) >> 1;
        return 2;
    }

    // Canonical order of the interpolation sums (every kernel uses it, so all
    // of them round alike): for each contributing coarse row Y_b, first the z
    // sum t_b(X) = sum_a w_Z e_c(X, Y_b, Z_a) over the interior planes Z_a,
    // then s(X) = sum_b w_Y t_b(X), then the x weights.  The weights are
    // powers of two, and scaling by a power of two commutes with rounding
    // (away from the underflow range), so a kernel may also form the plain
    // sums in this order and apply the product of the weights once.
    // rowsum: s(X) for X = x0/2 .. x0/2 + V/2 (the last may be the ghost Pc).
    template <int D, int V> __device__ __forceinline__ void rowsum(int x0, int y, int z, PA (&s)[V / 2 + 1]) const {
        constexpr int H = V / 2;
        Grid<D> gc{Pc};
#pragma unroll
        for (int j = 0; j <= H; ++j) s[j] = PA(0);
        int Zs[2], Ys[2] = {0, 0};
        const int nz = split(z, Zs);
        const int ny = D == 3 ? split(y, Ys) : 1;
        const PA wz = nz == 1 ? PA(1) : PA(0.5), wy = ny == 1 ? PA(1) : PA(0.5);
        const int X0 = x0 >> 1;
        for (int bb = 0; bb < ny; ++bb) {
            const int Y = D == 3 ? Ys[bb] : 0;
            PA t[H + 1];
#pragma unroll
            for (int j = 0; j <= H; ++j) t[j] = PA(0);
            if (!(D == 3 && (Y < 1 || Y >= Pc))) {
                for (int a = 0; a < nz; ++a) {
                    const int Z = Zs[a];
                    if (Z < 1 || Z >= Pc) continue;
                    const TC *base = ec + gc.at(X0, Y, Z);
                    PA v[H];
                    load_row<TC, H>(base, v);
#pragma unroll
                    for (int j = 0; j < H; ++j) t[j] += wz * v[j];
                    const PA last = (X0 + H < Pc) ? (PA)widen(base[H]) : PA(0);
                    t[H] += wz * last;
                }
            }
#pragma unroll
            for (int j = 0; j <= H; ++j) s[j] += wy * t[j];
        }
    }

    template <int D, int V> __device__ __forceinline__ void row(const Grid<D> &g, int x0, int y, int z, acc (&o)[V]) const {
        if (g.ghost_row(y, z)) {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = acc(0);
            return;
        }
        PA s[V / 2 + 1];
        rowsum<D, V>(x0, y, z, s);
        acc cv[V];
        load_row<TF, V>(c + g.at(x0, y, z), cv);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const PA p = (i & 1) ? PA(0.5) * (s[i >> 1] + s[(i >> 1) + 1]) : s[i >> 1];
            o[i] = round_to<TF>((PA)cv[i] + PA(4) * p);
        }
        if (x0 == 0) o[0] = acc(0);
    }

    // s(X) at one coarse X, in the canonical order
    template <int D> __device__ __forceinline__ PA colsum(int X, int y, int z) const {
        Grid<D> gc{Pc};
        PA s = PA(0);
        int Zs[2], Ys[2] = {0, 0};
        const int nz = split(z, Zs);
        const int ny = D == 3 ? split(y, Ys) : 1;
        const PA wz = nz == 1 ? PA(1) : PA(0.5), wy = ny == 1 ? PA(1) : PA(0.5);
        for (int bb = 0; bb < ny; ++bb) {
            const int Y = D == 3 ? Ys[bb] : 0;
            PA t = PA(0);
            if (X >= 1 && X < Pc && !(D == 3 && (Y < 1 || Y >= Pc))) {
                for (int a = 0; a < nz; ++a) {
                    const int Z = Zs[a];
                    if (Z < 1 || Z >= Pc) continue;
                    t += wz * (PA)widen(ec[gc.at(X, Y, Z)]);
                }
            }
            s += wy * t;
        }
        return s;
    }

    template <int D> __device__ __forceinline__ acc one(const Grid<D> &g, int x, int y, int z) const {
        if (x <= 0 || x >= g.P || g.ghost_row(y, z)) return acc(0);
        PA p;
        if ((x & 1) == 0) {
            p = colsum<D>(x >> 1, y, z);
        } else {
            p = PA(0.5) * (colsum<D>((x - 1) >> 1, y, z) + colsum<D>((x + 1) >> 1, y, z));
        }
        return round_to<TF>((PA)widen(c[g.at(x, y, z)]) + PA(4) * p);
    }
};

// ===========================================================================
// Emit policies: what a stencil kernel does with the centre values c and the
// neighbour sums nb of its row.
// ===========================================================================
struct NoState {};

// Damped-Jacobi sweep out = round_T(c + k (b - (2D c - nb))); optionally also
// stores the right-hand side it used (the scaled-and-cast residual).
template <class T, class R, bool WRITE_B> struct ESweep {
    typedef acc_t<T> A;
    typedef NoState State;
    R rhs;
    T *__restrict__ out;
    T *__restrict__ bout;
    A k;
    __device__ __forceinline__ void init(State &) const {}
    __device__ __forceinline__ void finish(State &, double *, long) const {}
    template <int D, int V>
    __device__ __forceinline__ void emit(const Grid<D> &g, State &, int x0, int y, int z, const A (&c)[V],
                                         const A (&nb)[V]) const {
        A b[V];
        rhs.template row<D, V>(g, x0, y, z, b);
        T o[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const A lc = fmaT<A>(A(2 * D), c[i], -nb[i]);
            o[i] = Store<T>::from_acc(fmaT<A>(k, b[i] - lc, c[i]));
        }
        if (x0 == 0) o[0] = Store<T>::from_acc(A(0));
        const size_t at = g.at(x0, y, z);
        store_row<T, V>(out + at, o);
        if (WRITE_B) {
            T bo[V];
#pragma unroll
            for (int i = 0; i < V; ++i) bo[i] = Store<T>::from_acc(b[i]);
            if (x0 == 0) bo[0] = Store<T>::from_acc(A(0));
            store_row<T, V>(bout + at, bo);
        }
    }
};

// Store the field itself (the first Jacobi iterate, or a correction without
// post-smoothing); optionally the right-hand side too.
template <class T, class R, bool WRITE_B> struct ECopy {
    typedef acc_t<T> A;
    typedef NoState State;
    R rhs;
    T *__restrict__ out;
    T *__restrict__ bout;
    __device__ __forceinline__ void init(State &) const {}
    __device__ __forceinline__ void finish(State &, double *, long) const {}
    template <int D, int V>
    __device__ __forceinline__ void emit(const Grid<D> &g, State &, int x0, int y, int z, const A (&c)[V],
                                         const A (&)[V]) const {
        T o[V];
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = Store<T>::from_acc(c[i]);
        if (x0 == 0) o[0] = Store<T>::from_acc(A(0));
        const size_t at = g.at(x0, y, z);
        store_row<T, V>(out + at, o);
        if (WRITE_B) {
            A b[V];
            rhs.template row<D, V>(g, x0, y, z, b);
            T bo[V];
#pragma unroll
            for (int i = 0; i < V; ++i) bo[i] = Store<T>::from_acc(b[i]);
            if (x0 == 0) bo[0] = Store<T>::from_acc(A(0));
            store_row<T, V>(bout + at, bo);
        }
    }
};

// Solution and residual update of Algorithm 2 in FP64 (grid-scaled c):
// u += alpha h^2 c,  r -= alpha (2D c - nb), plus per-block norm partials.
struct EOuter {
    typedef double A;
    struct State {
        double ss, mx;
    };
    double *__restrict__ R;
    double *__restrict__ U;
    const double *__restrict__ scal;
    double h2;
    double *__restrict__ part;
    __device__ __forceinline__ void init(State &s) const { s.ss = 0.0, s.mx = 0.0; }
    template <int D, int V>
    __device__ __forceinline__ void emit(const Grid<D> &g, State &st, int x0, int y, int z, const A (&c)[V],
                                         const A (&nb)[V]) const {
        const double a = scal[0];
        const double ah2 = a * h2;
        const size_t at = g.at(x0, y, z);
        double r[V], u[V];
        load_row<double, V>(R + at, r);
        load_row<double, V>(U + at, u);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const double lc = fmaT<double>(double(2 * D), c[i], -nb[i]);
            r[i] = fmaT<double>(-a, lc, r[i]);
            u[i] = fmaT<double>(ah2, c[i], u[i]);
        }
        if (x0 == 0) r[0] = 0.0, u[0] = 0.0;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            st.ss += r[i] * r[i];
            st.mx = nanmax(st.mx, fabs(r[i]));
        }
        store_row<double, V>(R + at, r);
        store_row<double, V>(U + at, u);
    }
    __device__ __forceinline__ void finish(State &s, double *lds, long pidx) const {
        block_reduce(s.ss, s.mx, lds);
        if (threadIdx.x == 0) {
            part[2 * pidx] = s.ss;
            part[2 * pidx + 1] = s.mx;
        }
    }
};

// ===========================================================================
// The z-marching stencil kernel.  Thread t of the grid owns x chunk
// (t mod P/V) of line (t div P/V); a line is a row y (3-D) of one z chunk, or
// one z chunk (2-D).  The neighbour sum is formed in the fixed order
// x-, x+, y-, y+, z-, z+ (2-D: x-, x+, then the two row neighbours).
// ===========================================================================
template <int D, int V, class F, class E>
__device__ __forceinline__ void stencil_body(const F &f, const E &e, int P, int zc, int nchunks, long blk,
                                             double *red, long pidx) {
    typedef typename F::acc A;
    const Grid<D> g{P};
    const int TXR = P / V;
    const int NY = D == 3 ? P : 1;
    const long t = blk * blockDim.x + threadIdx.x;
    const int xc = (int)(t % TXR);
    const long line = t / TXR;
    const int y = (int)(line % NY);
    const int chunk = (int)(line / NY);
    const bool active = chunk < nchunks && (D == 2 || y >= 1);
    typename E::State st;
    e.init(st);
    if (active) {
        const int z0 = 1 + chunk * zc;
        const int z1 = min(z0 + zc, P);
        const int x0 = xc * V;
        A cm[V], cc[V], cp[V];
        f.template row<D, V>(g, x0, y, z0 - 1, cm);
        f.template row<D, V>(g, x0, y, z0, cc);
        for (int z = z0; z < z1; ++z) {
            f.template row<D, V>(g, x0, y, z + 1, cp);
            A nb[V];
            const A xl = f.template one<D>(g, x0 - 1, y, z);
            const A xr = f.template one<D>(g, x0 + V, y, z);
#pragma unroll
            for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? cc[i - 1] : xl) + (i < V - 1 ? cc[i + 1] : xr);
            if constexpr (D == 3) {
                A ym[V], yp[V];
                f.template row<D, V>(g, x0, y - 1, z, ym);
                f.template row<D, V>(g, x0, y + 1, z, yp);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    nb[i] += ym[i];
                    nb[i] += yp[i];
                }
            }
#pragma unroll
            for (int i = 0; i < V; ++i) {
                nb[i] += cm[i];
                nb[i] += cp[i];
            }
            e.template emit<D, V>(g, st, x0, y, z, cc, nb);
#pragma unroll
            for (int i = 0; i < V; ++i) {
                cm[i] = cc[i];
                cc[i] = cp[i];
            }
        }
    }
    e.finish(st, red, pidx);
}

template <int D, int V, class F, class E>
__global__ __launch_bounds__(256) void k_stencil(F f, E e, int P, int zc, int nchunks, int xcd) {
    __shared__ double red[8];
    long blk = blockIdx.x;
    if (xcd) {
        // blocks are dealt round-robin to the 8 XCDs: give each XCD a
        // contiguous range of tiles so neighbouring rows share an L2
        const long nb = gridDim.x;
        blk = xcd_block(blk, nb);
    }
    stencil_body<D, V>(f, e, P, zc, nchunks, blk, red, (long)blockIdx.x);
}

// ===========================================================================
// Pipelined 3-D z-march with the field's current plane staged in LDS.
//
// A block owns TY output rows of full length P and a chunk of zc planes; its
// threads form TY + 2 row groups (the extra two produce the halo rows y0 - 1
// and y0 + TY).  Per plane, every row group evaluates the field once for its
// own row: the value stays in registers for the z-1 / z / z+1 queue and is
// written to one of two LDS plane buffers, from which the x and y neighbours
// are read after a barrier.  Global loads of the next plane are issued one
// iteration ahead ("fetch" into raw registers, "value" converts), so they are
// in flight across the barrier and the arithmetic.
//
// Policies (templated on V): a field provides Raw, fetch(), value() and the
// LDS storage type lds_t (field values are exactly representable in it); an
// emit provides Raw (per-row inputs of the output), fetch(), emit(), finish().
// ===========================================================================

// Stored array.
template <class T, class A, int V> struct PArr {
    typedef A acc;
    typedef T lds_t;
    typedef RawRow<T, V> Raw;
    const T *__restrict__ p;
    __device__ __forceinline__ void fetch(const Grid<3> &g, int x0, int y, int z, Raw &r) const {
        if (g.ghost_row(y, z)) {
            zero_row(r);
            return;
        }
        fetch_row<T, V>(p + g.at(x0, y, z), r);
    }
    __device__ __forceinline__ void value(const Raw &r, int, int, int, A (&o)[V], A (&)[V]) const {
        widen_row<T, V>(r, o);
    }
    static constexpr bool kStaged = false;
    __device__ __forceinline__ void bind_lds(unsigned char *, int, int, int) {}
    __device__ __forceinline__ void stage(int, int, int) const {}
};

// First Jacobi iterate round_T(k b) from a stored right-hand side; aux = b.
template <class T, int V> struct PJac0Arr {
    typedef acc_t<T> acc;
    typedef T lds_t;
    typedef RawRow<T, V> Raw;
    const T *__restrict__ b;
    acc k;
    __device__ __forceinline__ void fetch(const Grid<3> &g, int x0, int y, int z, Raw &r) const {
        if (g.ghost_row(y, z)) {
            zero_row(r);
            return;
        }
        fetch_row<T, V>(b + g.at(x0, y, z), r);
    }
    __device__ __forceinline__ void value(const Raw &r, int, int, int, acc (&o)[V], acc (&aux)[V]) const {
        widen_row<T, V>(r, aux);
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = round_to<T>(k * aux[i]);
    }
    static constexpr bool kStaged = false;
    __device__ __forceinline__ void bind_lds(unsigned char *, int, int, int) {}
    __device__ __forceinline__ void stage(int, int, int) const {}
};

// First Jacobi iterate from the scaled-and-cast FP64 residual; aux = b-hat.
template <class T, int V> struct PJac0Scaled {
    typedef acc_t<T> acc;
    typedef T lds_t;
    typedef RawRow<double, V> Raw;
    const double *__restrict__ r;
    const double *__restrict__ scal;  // scal[1] = 1/alpha
    acc k;
    __device__ __forceinline__ void fetch(const Grid<3> &g, int x0, int y, int z, Raw &rr) const {
        if (g.ghost_row(y, z)) {
            zero_row(rr);
            return;
        }
        fetch_row<double, V>(r + g.at(x0, y, z), rr);
    }
    __device__ __forceinline__ void value(const Raw &rr, int, int, int, acc (&o)[V], acc (&aux)[V]) const {
        const double inv = scal[1];
        double rv[V];
        widen_row<double, V>(rr, rv);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            aux[i] = widen(Store<T>::from_f64(rv[i] * inv));
            o[i] = round_to<T>(k * aux[i]);
        }
    }
    static constexpr bool kStaged = false;
    __device__ __forceinline__ void bind_lds(unsigned char *, int, int, int) {}
    __device__ __forceinline__ void stage(int, int, int) const {}
};

// Corrected correction round_TF(c + 4 P e_c); same arithmetic as FProl::row.
template <class TF, class TC, int V> struct PProl {
    typedef acc_t<TF> acc;
    typedef TF lds_t;
    typedef typename FProl<TF, TC>::PA PA;
    static constexpr int H = V / 2;
    struct Raw {
        RawRow<TF, V> c;
        RawRow<TC, H> seg[4];  // coarse row (Z_a, Y_b) at a * 2 + b
        TC last[4];
    };
    const TF *__restrict__ c;
    const TC *__restrict__ ec;
    int Pc;
    // Coarse rows (Z_a, Y_b) for a < nz, b < ny; a row on a ghost plane or
    // ghost row is fetched as zeros (it adds nothing to the sums).
    __device__ __forceinline__ void fetch(const Grid<3> &g, int x0, int y, int z, Raw &r) const {
        if (g.ghost_row(y, z)) {  // all zeros: the row's value is zero
            zero_row(r.c);
#pragma unroll
            for (int k = 0; k < 4; ++k) zero_row(r.seg[k]), r.last[k] = zero_of<TC>();
            return;
        }
        fetch_row<TF, V>(c + g.at(x0, y, z), r.c);
        const Grid<3> gc{Pc};
        int Zs[2], Ys[2];
        const int nz = FProl<TF, TC>::split(z, Zs);
        const int ny = FProl<TF, TC>::split(y, Ys);
        const int X0 = x0 >> 1;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
                const int idx = a * 2 + bb;
                if (a < nz && bb < ny) {
                    if (Zs[a] >= 1 && Zs[a] < Pc && Ys[bb] >= 1 && Ys[bb] < Pc) {
                        const TC *base = ec + gc.at(X0, Ys[bb], Zs[a]);
                        fetch_row<TC, H>(base, r.seg[idx]);
                        r.last[idx] = (X0 + H < Pc) ? base[H] : zero_of<TC>();
                    } else {
                        zero_row(r.seg[idx]);
                        r.last[idx] = zero_of<TC>();
                    }
                }
            }
        }
    }
    // The canonical sums with the weights applied once: S(X) = (e(Z_0, Y_0) +
    // e(Z_1, Y_0)) + (e(Z_0, Y_1) + e(Z_1, Y_1)) over the present terms, then
    // c + 4 w_Z w_Y S at even x and c + 4 w_Z w_Y (S(X) + S(X+1)) / 2 at odd x.
    // nz is the same for the whole block (one plane), ny for a whole row.
    __device__ __forceinline__ void value(const Raw &r, int x0, int y, int z, acc (&o)[V], acc (&)[V]) const {
        const int nz = (z & 1) ? 2 : 1;
        const int ny = (y & 1) ? 2 : 1;
        PA t[2][H + 1];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            if (bb < ny) {
                PA u[H];
                widen_row<TC, H>(r.seg[bb], u);
#pragma unroll
                for (int j = 0; j < H; ++j) t[bb][j] = u[j];
                t[bb][H] = (PA)widen(r.last[bb]);
                if (nz == 2) {
                    PA v[H];
                    widen_row<TC, H>(r.seg[2 + bb], v);
#pragma unroll
                    for (int j = 0; j < H; ++j) t[bb][j] += v[j];
                    t[bb][H] += (PA)widen(r.last[2 + bb]);
                }
            }
        }
        PA S[H + 1];
#pragma unroll
        for (int j = 0; j <= H; ++j) S[j] = ny == 2 ? t[0][j] + t[1][j] : t[0][j];
        const PA k0 = PA(4) * (nz == 2 ? PA(0.5) : PA(1)) * (ny == 2 ? PA(0.5) : PA(1));
        const PA k1 = PA(0.5) * k0;
        acc cv[V];
        widen_row<TF, V>(r.c, cv);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const PA q = (i & 1) ? S[i >> 1] + S[(i >> 1) + 1] : S[i >> 1];
            o[i] = round_to<TF>((PA)cv[i] + ((i & 1) ? k1 : k0) * q);
        }
        if (x0 == 0) o[0] = acc(0);
    }
    static constexpr bool kStaged = false;
    __device__ __forceinline__ void bind_lds(unsigned char *, int, int, int) {}
    __device__ __forceinline__ void stage(int, int, int) const {}
};

// Corrected correction with the coarse data staged in LDS: for every fine
// plane z the block first writes the z-interpolated coarse rows
// Ez(X, Y) = sum_a w_Z e_c(X, Y, Z_a) it needs (rows Ylo .. Ylo+NYc-1, all X,
// ghost rows and columns zero) into one of three LDS slots, two planes ahead;
// a fine row then reads one or two of those rows.  Same sums, same order as
// FProl, so the result is identical.
template <class TF, class TC, int V> struct PProlS {
    typedef acc_t<TF> acc;
    typedef TF lds_t;
    typedef typename FProl<TF, TC>::PA PA;
    static constexpr int H = V / 2;
    static constexpr bool kStaged = true;
    typedef RawRow<TF, V> Raw;
    const TF *__restrict__ c;
    const TC *__restrict__ ec;
    int Pc;
    PA *ez;        // [3][NYc][RSx]
    int Ylo, NYc, RSx;
    __device__ __forceinline__ static int ez_rows(int y0, int TY) { return (y0 + TY + 1) / 2 - (y0 - 1) / 2 + 1; }
    __device__ __forceinline__ void bind_lds(unsigned char *p, int y0, int TY, int) {
        ez = reinterpret_cast<PA *>(p);
        Ylo = (y0 - 1) / 2;
        NYc = ez_rows(y0, TY);
        RSx = Pc + 4;
    }
    // Staging is software-pipelined: stage_fetch loads the coarse values a
    // thread needs for Ez of fine plane z into registers (elements
    // e = tid + k * nthr of the slot, k < KS), stage_store combines and
    // writes them into slot z mod 3 one iteration later.
    static constexpr int KS = 4;
    struct Stage {
        TC v[KS][2];
    };
    __device__ __forceinline__ void stage_fetch(int z, int tid, int nthr, Stage &S) const {
        const Grid<3> gc{Pc};
        int Zs[2] = {0, 0};
        const int nz = FProl<TF, TC>::split(z, Zs);
        const bool plane_ok = z >= 1 && z < 2 * Pc;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int e = tid + k * nthr;
            const int r = e / RSx, X = e - r * RSx;
            const int Y = Ylo + r;
            const bool ok = plane_ok && e < NYc * RSx && X >= 1 && X < Pc && Y >= 1 && Y < Pc;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int Z = Zs[a];
                S.v[k][a] = (ok && a < nz && Z >= 1 && Z < Pc) ? ec[gc.at(X, Y, Z)] : zero_of<TC>();
            }
        }
    }
    __device__ __forceinline__ void stage_store(int z, int tid, int nthr, const Stage &S) const {
        int Zs[2] = {0, 0};
        const int nz = FProl<TF, TC>::split(z, Zs);
        const PA wz = nz == 1 ? PA(1) : PA(0.5);
        PA *dst = ez + (size_t)(z % 3) * NYc * RSx;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int e = tid + k * nthr;
            if (e < NYc * RSx) {
                PA t = PA(0);
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    if (a < nz && Zs[a] >= 1 && Zs[a] < Pc) t += wz * (PA)widen(S.v[k][a]);
                dst[e] = t;
            }
        }
    }
    __device__ __forceinline__ void stage(int z, int tid, int nthr) const {
        Stage S;
        stage_fetch(z, tid, nthr, S);
        stage_store(z, tid, nthr, S);
    }
    __device__ __forceinline__ void fetch(const Grid<3> &g, int x0, int y, int z, Raw &r) const {
        if (g.ghost_row(y, z)) {
            zero_row(r);
            return;
        }
        fetch_row<TF, V>(c + g.at(x0, y, z), r);
    }
    __device__ __forceinline__ void value(const Raw &r, int x0, int y, int z, acc (&o)[V], acc (&)[V]) const {
        const Grid<3> g{2 * Pc};
        if (g.ghost_row(y, z)) {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = acc(0);
            return;
        }
        int Ys[2];
        const int ny = FProl<TF, TC>::split(y, Ys);
        const PA wy = ny == 1 ? PA(1) : PA(0.5);
        const PA *slot = ez + (size_t)(z % 3) * NYc * RSx;
        const int X0 = x0 >> 1;
        PA s[H + 1];
#pragma unroll
        for (int j = 0; j <= H; ++j) s[j] = PA(0);
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            if (bb < ny) {
                const PA *row = slot + (size_t)(Ys[bb] - Ylo) * RSx + X0;
                PA t[H];
                load_row<PA, H>(row, t);
#pragma unroll
                for (int j = 0; j < H; ++j) s[j] += wy * t[j];
                s[H] += wy * row[H];
            }
        }
        acc cv[V];
        widen_row<TF, V>(r, cv);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const PA p = (i & 1) ? PA(0.5) * (s[i >> 1] + s[(i >> 1) + 1]) : s[i >> 1];
            o[i] = round_to<TF>((PA)cv[i] + PA(4) * p);
        }
        if (x0 == 0) o[0] = acc(0);
    }
};

// Damped-Jacobi output; the right-hand side is the field's aux (first
// pre-smoothing) or a stored array fetched one plane ahead.
template <class T, int V, bool RHS_AUX, bool WRITE_B> struct PSweep {
    typedef acc_t<T> A;
    typedef NoState State;
    typedef RawRow<T, RHS_AUX ? 2 : V> Raw;
    const T *__restrict__ b;
    T *__restrict__ out;
    T *__restrict__ bout;
    A k;
    __device__ __forceinline__ void init(State &) const {}
    __device__ __forceinline__ void finish(State &, double *, long) const {}
    __device__ __forceinline__ void fetch(const Grid<3> &g, int x0, int y, int z, Raw &r) const {
        if constexpr (!RHS_AUX) fetch_row<T, V>(b + g.at(x0, y, z), r);
    }
    __device__ __forceinline__ void emit(const Grid<3> &g, State &, int x0, int y, int z, const A (&c)[V],
                                         const A (&nb)[V], const A (&aux)[V], const Raw &r) const {
        T o[V];
        A bv[V];
        if constexpr (!RHS_AUX) widen_row<T, V>(r, bv);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const A bi = RHS_AUX ? aux[i] : bv[i];
            const A lc = fmaT<A>(A(6), c[i], -nb[i]);
            o[i] = Store<T>::from_acc(fmaT<A>(k, bi - lc, c[i]));
        }
        if (x0 == 0) o[0] = zero_of<T>();
        const size_t at = g.at(x0, y, z);
        store_row<T, V>(out + at, o);
        if constexpr (WRITE_B) {
            T bo[V];
#pragma unroll
            for (int i = 0; i < V; ++i) bo[i] = Store<T>::from_acc(aux[i]);
            if (x0 == 0) bo[0] = zero_of<T>();
            store_row<T, V>(bout + at, bo);
        }
    }
};

// Refinement update (FP64), R and U rows fetched one plane ahead.
template <int V> struct POuter {
    typedef double A;
    struct State {
        double ss, mx;
    };
    struct Raw {
        RawRow<double, V> r, u;
    };
    double *__restrict__ R;
    double *__restrict__ U;
    const double *__restrict__ scal;
    double h2;
    double *__restrict__ part;
    __device__ __forceinline__ void init(State &s) const { s.ss = 0.0, s.mx = 0.0; }
    __device__ __forceinline__ void fetch(const Grid<3> &g, int x0, int y, int z, Raw &r) const {
        const size_t at = g.at(x0, y, z);
        fetch_row<double, V>(R + at, r.r);
        fetch_row<double, V>(U + at, r.u);
    }
    __device__ __forceinline__ void emit(const Grid<3> &g, State &st, int x0, int y, int z, const A (&c)[V],
                                         const A (&nb)[V], const A (&)[V], const Raw &rw) const {
        const double a = scal[0];
        const double ah2 = a * h2;
        double r[V], u[V];
        widen_row<double, V>(rw.r, r);
        widen_row<double, V>(rw.u, u);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const double lc = fmaT<double>(6.0, c[i], -nb[i]);
            r[i] = fmaT<double>(-a, lc, r[i]);
            u[i] = fmaT<double>(ah2, c[i], u[i]);
        }
        if (x0 == 0) r[0] = 0.0, u[0] = 0.0;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            st.ss += r[i] * r[i];
            st.mx = nanmax(st.mx, fabs(r[i]));
        }
        const size_t at = g.at(x0, y, z);
        store_row<double, V>(R + at, r);
        store_row<double, V>(U + at, u);
    }
    __device__ __forceinline__ void finish(State &s, double *lds, long pidx) const {
        block_reduce(s.ss, s.mx, lds);
        if (threadIdx.x == 0) {
            part[2 * pidx] = s.ss;
            part[2 * pidx + 1] = s.mx;
        }
    }
};

template <class F, class = void> struct StageOf {
    struct type {};
};
template <class F> struct StageOf<F, typename std::enable_if<F::kStaged>::type> {
    typedef typename F::Stage type;
};

// DP: field and emit rows of DP planes ahead are in flight while a plane is
// computed (the loads for plane z + 1 + DP are issued in iteration z).
// One tile (blk = y tile + ytiles * z chunk) of the LDS-plane march; pidx is
// the index of the block's norm partial.  Called by every thread of the block.
template <int V, class F, class E, int DP>
__device__ __forceinline__ void march_body(const F &f_in, const E &e, int P, int TY, int zc, int ytiles, int blk,
                                           long pidx, unsigned char *smem_raw, double *red) {
    typedef typename F::acc A;
    typedef typename F::lds_t LT;
    typedef LdsRun<LT, V> LR;  // LDS rows, chunk-major
    LT *lds = reinterpret_cast<LT *>(smem_raw);
    const Grid<3> g{P};
    const int TXR = P / V;
    const int G = TY + 2;
    const int yt = blk % ytiles, zch = blk / ytiles;
    const int y0 = 1 + yt * TY;
    const int z0 = 1 + zch * zc;
    const int z1 = min(z0 + zc, P);
    const int xc = threadIdx.x % TXR, gi = threadIdx.x / TXR;
    const int y = y0 - 1 + gi;
    const bool out_row = gi >= 1 && gi <= TY && y <= P - 1;
    const int x0 = xc * V;
    const size_t slot = (size_t)G * P;
    typename E::State st;
    e.init(st);
    typename F::Raw fr, fq[DP];
    typename E::Raw eq[DP];
    A cm[V], cc[V], cp[V], ac[V], ap[V];
    F f = f_in;
    const int nthr = blockDim.x;
    typename StageOf<F>::type S;
    if constexpr (F::kStaged) {
        f.bind_lds(smem_raw + 2 * slot * sizeof(LT), y0, TY, 0);
        f.stage(z0 - 1, threadIdx.x, nthr);
        f.stage(z0, threadIdx.x, nthr);
        f.stage(z0 + 1, threadIdx.x, nthr);
        f.stage_fetch(z0 + 2, threadIdx.x, nthr, S);
        __syncthreads();
    }
    f.fetch(g, x0, y, z0 - 1, fr);
    f.value(fr, x0, y, z0 - 1, cm, ac);
    f.fetch(g, x0, y, z0, fr);
    f.value(fr, x0, y, z0, cc, ac);
    {
        LT t[V];
#pragma unroll
        for (int i = 0; i < V; ++i) t[i] = store_as<LT>(cc[i]);
        LR::store(lds + (size_t)gi * P, xc, TXR, t);
    }
    // queues: fq[d] holds field plane z + 1 + d, eq[d] the emit rows of plane z + d
#pragma unroll
    for (int d = 0; d < DP; ++d) {
        if (z0 + 1 + d <= z1) f.fetch(g, x0, y, z0 + 1 + d, fq[d]);
        if (out_row && z0 + d < z1) e.fetch(g, x0, y, z0 + d, eq[d]);
    }
    if constexpr (F::kStaged) __syncthreads();  // prologue reads of the staged slots are done
    for (int z = z0; z < z1; ++z) {
        const int it = z - z0;
        f.value(fq[0], x0, y, z + 1, cp, ap);
        if constexpr (F::kStaged) {
            f.stage_store(z + 2, threadIdx.x, nthr, S);
            if (z + 3 <= z1) f.stage_fetch(z + 3, threadIdx.x, nthr, S);
        }
        const typename E::Raw ecur = eq[0];
#pragma unroll
        for (int d = 0; d + 1 < DP; ++d) {
            fq[d] = fq[d + 1];
            eq[d] = eq[d + 1];
        }
        if (z + 1 + DP <= z1) f.fetch(g, x0, y, z + 1 + DP, fq[DP - 1]);
        if (out_row && z + DP < z1) e.fetch(g, x0, y, z + DP, eq[DP - 1]);
        __syncthreads();
        if (out_row) {
            const LT *S = lds + (size_t)(it & 1) * slot;
            const LT *row = S + (size_t)gi * P;
            A nb[V];
            const A xl = x0 > 0 ? (A)widen(LR::left_of(row, xc, TXR)) : A(0);
            const A xr = x0 + V < P ? (A)widen(LR::right_of(row, xc, TXR)) : A(0);
#pragma unroll
            for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? cc[i - 1] : xl) + (i < V - 1 ? cc[i + 1] : xr);
            A ym[V], yp[V];
            LR::load(row - P, xc, TXR, ym);
            LR::load(row + P, xc, TXR, yp);
#pragma unroll
            for (int i = 0; i < V; ++i) {
                nb[i] += ym[i];
                nb[i] += yp[i];
                nb[i] += cm[i];
                nb[i] += cp[i];
            }
            e.emit(g, st, x0, y, z, cc, nb, ac, ecur);
        }
        {
            LT t[V];
#pragma unroll
            for (int i = 0; i < V; ++i) t[i] = store_as<LT>(cp[i]);
            LR::store(lds + (size_t)((it + 1) & 1) * slot + (size_t)gi * P, xc, TXR, t);
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            cm[i] = cc[i];
            cc[i] = cp[i];
            ac[i] = ap[i];
        }
    }
    e.finish(st, red, pidx);
}

template <int V, class F, class E, int DP = 1>
__global__ __launch_bounds__(1024) void k_march(F f_in, E e, int P, int TY, int zc, int ytiles, int xcd) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[32];
    int blk = blockIdx.x;
    if (xcd) {
        // blocks are dealt round-robin to the 8 XCDs: give each XCD a
        // contiguous range of tiles so neighbouring rows share an L2
        const int nb = gridDim.x;
        blk = xcd_block(blk, nb);
    }
    march_body<V, F, E, DP>(f_in, e, P, TY, zc, ytiles, blk, (long)blockIdx.x, smem_raw, red);
}

// ===========================================================================
// Residual + full-weighting restriction + cast (the residual transfer of
// Algorithm 1).  A block
// owns `tyc` coarse rows (3-D) and `zcc` coarse planes.  Its threads first act
// as fine-row threads: 2 tyc + 1 fine rows (2-D: one), each thread V fine x
// values, marching the fine planes 2Z0-1 .. 2Z1-1 and writing the fine
// residual b - L c of every plane into an LDS row buffer (double-buffered).
// After a barrier the first tyc * P/V threads act as coarse threads with V/2
// coarse x values each: they apply the x and y weights (1/4, 1/2, 1/4) from
// LDS and accumulate the z weights in registers across the march.
// ===========================================================================
template <int D, int V, class TF, class TC>
__device__ __forceinline__ void restrict_body(const TF *__restrict__ b, const TF *__restrict__ c,
                                              TC *__restrict__ bc, int P, int tyc, int zcc, int ytiles, int blk,
                                              unsigned char *smem_raw) {
    typedef acc_t<TF> A;
    constexpr int VC = V / 2;
    A *rs = reinterpret_cast<A *>(smem_raw);
    const int Pc = P >> 1;
    const int TXR = P / V;
    const int G = D == 3 ? 2 * tyc + 1 : 1;
    const Grid<D> g{P};
    const Grid<D> gc{Pc};
    const int ytile = blk % ytiles, zch = blk / ytiles;
    const int Y0 = D == 3 ? 1 + ytile * tyc : 0;
    const int Z0 = 1 + zch * zcc;
    const int Z1 = min(Z0 + zcc, Pc);
    const int tid = threadIdx.x;
    const int xc = tid % TXR, gi = tid / TXR;
    const bool fine_active = gi < G;
    const int y = D == 3 ? 2 * Y0 - 1 + gi : 0;
    const bool rowok = fine_active && !(D == 3 && y >= P);
    const int x0 = xc * V;
    const bool coarse_active = D == 3 ? (gi < tyc && Y0 + gi < Pc) : (gi == 0);
    const int Yc = D == 3 ? Y0 + gi : 0;
    const int X0 = xc * VC;
    const FArr<TF, A> cf{c};
    const FArr<TF, A> bf{b};
    A acc[VC];
#pragma unroll
    for (int j = 0; j < VC; ++j) acc[j] = A(0);
    const int zf0 = 2 * Z0 - 1, zf1 = 2 * Z1 - 1;
    A cm[V], cc[V], cp[V];
    if (rowok) {
        cf.template row<D, V>(g, x0, y, zf0 - 1, cm);
        cf.template row<D, V>(g, x0, y, zf0, cc);
    }
    for (int zf = zf0; zf <= zf1; ++zf) {
        A *buf = rs + (size_t)((zf - zf0) & 1) * G * P;
        if (fine_active) {
            A r[V];
            if (rowok) {
                cf.template row<D, V>(g, x0, y, zf + 1, cp);
                A nb[V];
                const A xl = cf.template one<D>(g, x0 - 1, y, zf);
                const A xr = cf.template one<D>(g, x0 + V, y, zf);
#pragma unroll
                for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? cc[i - 1] : xl) + (i < V - 1 ? cc[i + 1] : xr);
                if constexpr (D == 3) {
                    A ym[V], yp[V];
                    cf.template row<D, V>(g, x0, y - 1, zf, ym);
                    cf.template row<D, V>(g, x0, y + 1, zf, yp);
#pragma unroll
                    for (int i = 0; i < V; ++i) {
                        nb[i] += ym[i];
                        nb[i] += yp[i];
                    }
                }
                A bb[V];
                bf.template row<D, V>(g, x0, y, zf, bb);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    nb[i] += cm[i];
                    nb[i] += cp[i];
                    r[i] = bb[i] - fmaT<A>(A(2 * D), cc[i], -nb[i]);
                }
                if (x0 == 0) r[0] = A(0);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    cm[i] = cc[i];
                    cc[i] = cp[i];
                }
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) r[i] = A(0);
            }
            A *dst = buf + (size_t)gi * P + x0;
#pragma unroll
            for (int i = 0; i < V; ++i) dst[i] = r[i];
        }
        __syncthreads();
        if (coarse_active) {
            const bool last_of_z = zf > zf0 && ((zf - zf0) & 1) == 0;  // zf = 2Z + 1
            TC out[VC];
#pragma unroll
            for (int j = 0; j < VC; ++j) {
                const int X = X0 + j;
                A q = A(0);
                if (X >= 1) {
                    if constexpr (D == 3) {
                        A rsum[3];
#pragma unroll
                        for (int oy = 0; oy < 3; ++oy) {
                            const A *row = buf + (size_t)(2 * gi + oy) * P;
                            rsum[oy] = A(0.25) * (row[2 * X - 1] + row[2 * X + 1]) + A(0.5) * row[2 * X];
                        }
                        q = A(0.25) * (rsum[0] + rsum[2]) + A(0.5) * rsum[1];
                    } else {
                        const A *row = buf;
                        q = A(0.25) * (row[2 * X - 1] + row[2 * X + 1]) + A(0.5) * row[2 * X];
                    }
                }
                if (zf == zf0) {
                    acc[j] = A(0.25) * q;
                } else if (!last_of_z) {
                    acc[j] += A(0.5) * q;
                } else {
                    const A v = acc[j] + A(0.25) * q;
                    out[j] = store_as<TC>(v);
                    acc[j] = A(0.25) * q;
                }
            }
            if (last_of_z) {
                if (X0 == 0) out[0] = store_as<TC>(A(0));
                const int Z = (zf - 1) >> 1;
                store_row<TC, VC>(bc + gc.at(X0, Yc, Z), out);
            }
        }
    }
}

template <int D, int V, class TF, class TC>
__global__ __launch_bounds__(1024) void k_restrict(const TF *__restrict__ b, const TF *__restrict__ c,
                                                   TC *__restrict__ bc, int P, int tyc, int zcc, int ytiles) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    restrict_body<D, V, TF, TC>(b, c, bc, P, tyc, zcc, ytiles, blockIdx.x, smem_raw);
}

// ===========================================================================
// Pipelined residual + restriction.  A block owns tyc coarse rows and zcc
// coarse planes.  Its threads form G = 2 tyc + 3 fine row groups: the fine
// rows 2Y0-2 .. 2Y0+2tyc whose correction values the residual rows
// 2Y0-1 .. 2Y0+2tyc-1 need.  Per fine plane the correction plane goes through a
// double-buffered LDS slot (as in k_march, with the next plane prefetched),
// every residual row group writes b - L c into a double-buffered LDS row
// buffer, and after the next barrier the first tyc * P/V threads combine three
// residual rows with the x and y weights and accumulate the z weights of the
// coarse plane in registers.  One barrier per fine plane.
// ===========================================================================
// XSH: the fine threads also apply the x weights, taking the residual at
// x0 - 1 from the previous lane by a wave shuffle (needs P/V <= 64, so a
// grid row never straddles two waves); the LDS row buffer then holds the
// x-restricted values, P/2 per row, and the coarse threads read VC of them
// per row as one vector.
// DP: planes of c and b in flight ahead of the plane being processed (the
// loads for plane zf + 1 + DP are issued while plane zf is computed).
template <int V, class TF, class TC, bool XSH, int DP>
__device__ __forceinline__ void restrict2_body(const TF *__restrict__ b, const TF *__restrict__ c,
                                               TC *__restrict__ bc, int P, int tyc, int zcc, int ytiles, int blk,
                                               unsigned char *smem_raw) {
    typedef acc_t<TF> A;
    constexpr int VC = V / 2;
    const int G = 2 * tyc + 3, R = 2 * tyc + 1;
    const int RW = XSH ? P / 2 : P;                                             // r row width
    TF *cs = reinterpret_cast<TF *>(smem_raw);                                  // [2][G][P]
    A *rs = reinterpret_cast<A *>(smem_raw + 2 * (size_t)G * P * sizeof(TF));   // [2][R][RW]
    const int Pc = P >> 1;
    const int TXR = P / V;
    const Grid<3> g{P};
    const Grid<3> gc{Pc};
    const int ytile = blk % ytiles, zch = blk / ytiles;
    const int Y0 = 1 + ytile * tyc;
    const int Z0 = 1 + zch * zcc;
    const int Z1 = min(Z0 + zcc, Pc);
    const int tid = threadIdx.x;
    const int xc = tid % TXR, gi = tid / TXR;
    const int y = 2 * Y0 - 2 + gi;
    const bool res_row = gi >= 1 && gi <= G - 2 && y <= P - 1;
    const int x0 = xc * V;
    const bool coarse = gi < tyc && Y0 + gi < Pc;
    const int Yc = Y0 + gi;
    const int X0 = xc * VC;
    const PArr<TF, A, V> f{c};
    const size_t cslot = (size_t)G * P, rslot = (size_t)R * RW;
    const int zf0 = 2 * Z0 - 1, zf1 = 2 * Z1 - 1;
    typename PArr<TF, A, V>::Raw fr, fq[DP];
    RawRow<TF, V> braw, bq[DP];
    A cm[V], cc[V], cp[V], dummy[V];
    A acc[VC];
#pragma unroll
    for (int j = 0; j < VC; ++j) acc[j] = A(0);
    f.fetch(g, x0, y, zf0 - 1, fr);
    f.value(fr, x0, y, zf0 - 1, cm, dummy);
    f.fetch(g, x0, y, zf0, fr);
    f.value(fr, x0, y, zf0, cc, dummy);
    {
        TF t[V];
#pragma unroll
        for (int i = 0; i < V; ++i) t[i] = store_as<TF>(cc[i]);
        store_row<TF, V>(cs + (size_t)gi * P + x0, t);
    }
    // queues: fq[d] holds c plane zf + 1 + d, bq[d] holds b plane zf + d
#pragma unroll
    for (int d = 0; d < DP; ++d) {
        if (zf0 + 1 + d <= zf1 + 1) f.fetch(g, x0, y, zf0 + 1 + d, fq[d]);
        if (res_row && zf0 + d <= zf1) fetch_row<TF, V>(b + g.at(x0, y, zf0 + d), bq[d]);
    }

    // coarse step: fold the residual rows of fine plane zf (in slot s) into acc
    auto coarse_step = [&](int zf, int s) {
        const A *rb = rs + (size_t)s * rslot;
        const int j = zf - zf0;
        const bool last_of_z = j > 0 && (j & 1) == 0;  // zf = 2Z + 1
        TC out[VC];
        A xs[3][VC];
        if constexpr (XSH) {
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) load_row<A, VC>(rb + (size_t)(2 * gi + oy) * RW + X0, xs[oy]);
        }
#pragma unroll
        for (int jx = 0; jx < VC; ++jx) {
            const int X = X0 + jx;
            A q = A(0);
            if (X >= 1) {
                A rsum[3];
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
                    if constexpr (XSH) {
                        rsum[oy] = xs[oy][jx];
                    } else {
                        const A *row = rb + (size_t)(2 * gi + oy) * P;
                        rsum[oy] = A(0.25) * (row[2 * X - 1] + row[2 * X + 1]) + A(0.5) * row[2 * X];
                    }
                }
                q = A(0.25) * (rsum[0] + rsum[2]) + A(0.5) * rsum[1];
            }
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

    A rkeep[V];
    for (int zf = zf0; zf <= zf1; ++zf) {
        const int it = zf - zf0;
#pragma unroll
        for (int i = 0; i < V; ++i) rkeep[i] = A(0);
        f.value(fq[0], x0, y, zf + 1, cp, dummy);
        braw = bq[0];
#pragma unroll
        for (int d = 0; d + 1 < DP; ++d) {
            fq[d] = fq[d + 1];
            bq[d] = bq[d + 1];
        }
        if (zf + 1 + DP <= zf1 + 1) f.fetch(g, x0, y, zf + 1 + DP, fq[DP - 1]);
        if (res_row && zf + DP <= zf1) fetch_row<TF, V>(b + g.at(x0, y, zf + DP), bq[DP - 1]);
        __syncthreads();
        if (coarse && it > 0) coarse_step(zf - 1, (it - 1) & 1);
        if (res_row) {
            const TF *row = cs + (size_t)(it & 1) * cslot + (size_t)gi * P;
            A nb[V];
            const A xl = x0 > 0 ? (A)widen(row[x0 - 1]) : A(0);
            const A xr = x0 + V < P ? (A)widen(row[x0 + V]) : A(0);
#pragma unroll
            for (int i = 0; i < V; ++i) nb[i] = (i > 0 ? cc[i - 1] : xl) + (i < V - 1 ? cc[i + 1] : xr);
            A ym[V], yp[V];
            load_row<TF, V>(row - P + x0, ym);
            load_row<TF, V>(row + P + x0, yp);
            A r[V], bv[V];
            widen_row<TF, V>(braw, bv);
#pragma unroll
            for (int i = 0; i < V; ++i) {
                nb[i] += ym[i];
                nb[i] += yp[i];
                nb[i] += cm[i];
                nb[i] += cp[i];
                r[i] = bv[i] - fmaT<A>(A(6), cc[i], -nb[i]);
            }
            if (x0 == 0) r[0] = A(0);
            if constexpr (!XSH) {
                A *dst = rs + (size_t)(it & 1) * rslot + (size_t)(gi - 1) * P + x0;
#pragma unroll
                for (int i = 0; i < V; ++i) dst[i] = r[i];
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) rkeep[i] = r[i];
            }
        } else if (!XSH && gi >= 1 && gi <= G - 2) {
            // residual rows past the last interior row are zero
            A *dst = rs + (size_t)(it & 1) * rslot + (size_t)(gi - 1) * P + x0;
#pragma unroll
            for (int i = 0; i < V; ++i) dst[i] = A(0);
        }
        if constexpr (XSH) {
            // x weights in the fine thread: coarse X = x0/2 + j takes fine
            // 2X-1, 2X, 2X+1 = x0+2j-1 .. x0+2j+1; x0-1 comes from the previous lane
            const A left_in = __shfl_up(rkeep[V - 1], 1, 64);
            const A left = x0 > 0 ? left_in : A(0);
            A xq[VC];
#pragma unroll
            for (int j = 0; j < VC; ++j) {
                const A lm = j > 0 ? rkeep[2 * j - 1] : left;
                xq[j] = A(0.25) * (lm + rkeep[2 * j + 1]) + A(0.5) * rkeep[2 * j];
            }
            if (x0 == 0) xq[0] = A(0);
            if (gi >= 1 && gi <= G - 2) store_row<A, VC>(rs + (size_t)(it & 1) * rslot + (size_t)(gi - 1) * RW + (x0 >> 1), xq);
        }
        {
            TF t[V];
#pragma unroll
            for (int i = 0; i < V; ++i) t[i] = store_as<TF>(cp[i]);
            store_row<TF, V>(cs + (size_t)((it + 1) & 1) * cslot + (size_t)gi * P + x0, t);
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            cm[i] = cc[i];
            cc[i] = cp[i];
        }
    }
    __syncthreads();
    if (coarse) coarse_step(zf1, (zf1 - zf0) & 1);
}

template <int V, class TF, class TC, bool XSH, int DP = 1>
__global__ __launch_bounds__(1024) void k_restrict2(const TF *__restrict__ b, const TF *__restrict__ c,
                                                    TC *__restrict__ bc, int P, int tyc, int zcc, int ytiles,
                                                    int xcd) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int blk = blockIdx.x;
    if (xcd) {
        const int nb = gridDim.x;
        blk = xcd_block(blk, nb);
    }
    restrict2_body<V, TF, TC, XSH, DP>(b, c, bc, P, tyc, zcc, ytiles, blk, smem_raw);
}

// Base level: the single interior point of an n = 1 grid (P = 2) at (1,1[,1]).
template <int D, class T> __global__ void k_coarse(const T *__restrict__ b, T *__restrict__ c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int i = D == 3 ? 7 : 3;
        typedef acc_t<T> A;
        c[i] = Store<T>::from_acc(widen(b[i]) / A(2 * D));
    }
}

// r = b - A U with the FP64 operator (2D u - nb) / h^2.  One wave per grid row
// (grid-stride over rows), consecutive lanes on consecutive x, so both the
// dense arrays and the padded ones are read and written coalesced.
template <int D>
__global__ __launch_bounds__(256) void k_resid_rows(const double *__restrict__ b, const double *__restrict__ U,
                                                    double *__restrict__ R, double *__restrict__ uout, int n, int P,
                                                    double inv_h2, double *__restrict__ part) {
    __shared__ double red[8];
    const Grid<D> g{P};
    const size_t plane = D == 3 ? (size_t)P * P : (size_t)P;
    const long rows = D == 3 ? (long)n * n : (long)n;
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    double ss = 0.0, mx = 0.0;
    for (long row = wave; row < rows; row += nwaves) {
        int y = 0, z;
        if (D == 3) {
            y = (int)(row % n) + 1;
            z = (int)(row / n) + 1;
        } else {
            z = (int)row + 1;
        }
        const size_t dbase = (size_t)row * n;
        const size_t pbase = g.at(1, y, z);
        for (int x = lane; x < n; x += 64) {
            const size_t p = pbase + x;
            double r = b[dbase + x];
            if (U) {
                double nb = U[p - 1] + U[p + 1];
                if (D == 3) {
                    nb += U[p - P];
                    nb += U[p + P];
                }
                nb += U[p - plane];
                nb += U[p + plane];
                r = r - (double(2 * D) * U[p] - nb) * inv_h2;
                if (uout) uout[dbase + x] = U[p];
            }
            if (R) R[p] = r;
            ss += r * r;
            mx = nanmax(mx, fabs(r));
        }
    }
    block_reduce(ss, mx, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss;
        part[2 * blockIdx.x + 1] = mx;
    }
}

// The same residual in 3-D, marching z: a tile is four consecutive rows y (one
// wave each, lane l on x = l + 64 k) and a chunk of zc planes.  Each lane keeps
// U of its points on planes z-1, z, z+1 in registers, so a plane of U is read
// from HBM once, when it becomes plane z+1; the y neighbours are the rows the
// waves beside it read at the same plane (cache hits), the x neighbours lie in
// the row the wave has just read.  Tiles are dealt to the XCDs in contiguous
// ranges (neighbouring y bands share an L2).  Blocks loop over tiles
// (gridDim.x may be below the tile count); one partial per block.
template <int KX>
__global__ __launch_bounds__(256) void k_resid_march(const double *__restrict__ b, const double *__restrict__ U,
                                                     double *__restrict__ R, double *__restrict__ uout, int n, int P,
                                                     double inv_h2, double *__restrict__ part, int ytiles, int zc,
                                                     int ntiles) {
    __shared__ double red[8];
    const Grid<3> g{P};
    const size_t plane = (size_t)P * P;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double ss = 0.0, mx = 0.0;
    for (int t = xcd_block(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x) {
        const int y = 1 + (t % ytiles) * 4 + w;
        const int z0 = 1 + (t / ytiles) * zc, z1 = min(z0 + zc, n + 1);
        if (y > n) continue;
        double um[KX], uc[KX], up[KX];
        // planes z0 - 1 and z0 (plane 0 is a zero ghost)
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            const int x = lane + 64 * k;
            const bool in = x < n;
            um[k] = in ? U[g.at(1 + x, y, z0 - 1)] : 0.0;
            uc[k] = in ? U[g.at(1 + x, y, z0)] : 0.0;
        }
        for (int z = z0; z < z1; ++z) {
            const size_t dbase = ((size_t)(z - 1) * n + (y - 1)) * n;
            const size_t pbase = g.at(1, y, z);
#pragma unroll
            for (int k = 0; k < KX; ++k) {
                const int x = lane + 64 * k;
                if (x < n) up[k] = U[pbase + plane + x];  // plane z+1 (plane n+1 is a zero ghost)
            }
#pragma unroll
            for (int k = 0; k < KX; ++k) {
                const int x = lane + 64 * k;
                if (x < n) {
                    const size_t p = pbase + x;
                    double nb = U[p - 1] + U[p + 1];
                    nb += U[p - P];
                    nb += U[p + P];
                    nb += um[k];
                    nb += up[k];
                    const double r = b[dbase + x] - (6.0 * uc[k] - nb) * inv_h2;
                    if (uout) uout[dbase + x] = uc[k];
                    if (R) R[p] = r;
                    ss += r * r;
                    mx = nanmax(mx, fabs(r));
                }
            }
#pragma unroll
            for (int k = 0; k < KX; ++k) {
                um[k] = uc[k];
                uc[k] = up[k];
            }
        }
    }
    block_reduce(ss, mx, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss;
        part[2 * blockIdx.x + 1] = mx;
    }
}

__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ part, int nparts, double *__restrict__ scal,
                                                  int scaling, int *__restrict__ ctr) {
    __shared__ double red[8];
    double s = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        s += part[2 * i];
        m = nanmax(m, part[2 * i + 1]);
    }
    block_reduce(s, m, red);
    if (threadIdx.x == 0) {
        double a = scaling ? ldexp(m, scaling - 1) : 1.0;
        if (!(a > 0.0) || a > 1.7e308) a = 1.0;
        scal[0] = a;
        scal[1] = 1.0 / a;
        scal[2] = sqrt(s);
        scal[3] = m;
        if (ctr) *ctr += 1;
    }
}

// u += a_j h^2 c_j over the postponed corrections in order; one thread per
// eight consecutive elements (the padded arrays have a multiple of 8).
// from_zero: u starts from 0 (the same sums as from a zero-filled U, which is
// then neither filled nor read).
template <class T>
__global__ __launch_bounds__(256) void k_defer_flush(const T *__restrict__ cd, size_t cstride,
                                                     const double *__restrict__ adef, int count, double h2,
                                                     double *__restrict__ U, size_t n8, int *__restrict__ ctr,
                                                     int from_zero) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += (size_t)gridDim.x * blockDim.x) {
        double u[8];
        if (from_zero) {
#pragma unroll
            for (int e = 0; e < 8; ++e) u[e] = 0.0;
        } else {
            load_row<double, 8>(U + 8 * i, u);
        }
        for (int j = 0; j < count; ++j) {
            const double ah2 = adef[j] * h2;
            double cv[8];
            load_row<T, 8>(cd + (size_t)j * cstride + 8 * i, cv);
#pragma unroll
            for (int e = 0; e < 8; ++e) u[e] = fmaT<double>(ah2, cv[e], u[e]);
        }
        store_row<double, 8>(U + 8 * i, u);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr = 0;
}

template <int D, class TS, class TD>
__global__ __launch_bounds__(256) void k_pack(const TS *__restrict__ src, TD *__restrict__ dst, int n, int P, long N) {
    const Grid<D> g{P};
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += (long)gridDim.x * blockDim.x) {
        const int x = (int)(idx % n) + 1;
        const long rest = idx / n;
        const int y = D == 3 ? (int)(rest % n) + 1 : 0;
        const int z = D == 3 ? (int)(rest / n) + 1 : (int)rest + 1;
        dst[g.at(x, y, z)] = Store<TD>::from_f64((double)widen(src[idx]));
    }
}

template <int D, class TS, class TD>
__global__ __launch_bounds__(256) void k_unpack(const TS *__restrict__ src, TD *__restrict__ dst, int n, int P, long N) {
    const Grid<D> g{P};
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += (long)gridDim.x * blockDim.x) {
        const int x = (int)(idx % n) + 1;
        const long rest = idx / n;
        const int y = D == 3 ? (int)(rest % n) + 1 : 0;
        const int z = D == 3 ? (int)(rest / n) + 1 : (int)rest + 1;
        dst[idx] = Store<TD>::from_f64((double)widen(src[g.at(x, y, z)]));
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(uint4 *__restrict__ p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Bandwidth probe: copy, read-only (sum kept live) or write-only passes over
// 16-byte lanes; each thread handles `per` consecutive lanes per grid sweep.
// 16-byte vector types for the probes' non-temporal accesses
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

template <bool NT, class V> __device__ __forceinline__ V ld_nt(const V *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class V> __device__ __forceinline__ void st_nt(V *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Bandwidth probe: copy, read-only (sum kept live) or write-only passes over
// 16-byte lanes in a grid-stride loop; NT: non-temporal loads and stores.
template <bool NT>
__global__ __launch_bounds__(256) void k_probe(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, size_t n16,
                                              int kind, unsigned *__restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        if (kind == 0) {
            st_nt<NT>(dst + i, ld_nt<NT>(src + i));
        } else if (kind == 1) {
            const u32x4 v = ld_nt<NT>(src + i);
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        } else {
            u32x4 v = {(uint32_t)i, 0u, 0u, 0u};
            st_nt<NT>(dst + i, v);
        }
    }
    if (kind == 1 && acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads live
}

// The refinement update's access mix: two FP64 arrays read and written, two
// FP16 arrays read, four elements per thread and step.  NTL / NTS:
// non-temporal loads / stores.
template <bool NTL, bool NTS>
__global__ __launch_bounds__(256) void k_probe_update(double *__restrict__ R, double *__restrict__ U,
                                                      const f16 *__restrict__ c, const f16 *__restrict__ b,
                                                      size_t n4) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        f64x2 *r2 = reinterpret_cast<f64x2 *>(R + 4 * i);
        f64x2 *u2 = reinterpret_cast<f64x2 *>(U + 4 * i);
        const f64x2 r0 = ld_nt<NTL>(r2), r1 = ld_nt<NTL>(r2 + 1);
        const f64x2 u0 = ld_nt<NTL>(u2), u1 = ld_nt<NTL>(u2 + 1);
        const f16x4 cv = ld_nt<NTL>(reinterpret_cast<const f16x4 *>(c + 4 * i));
        const f16x4 bv = ld_nt<NTL>(reinterpret_cast<const f16x4 *>(b + 4 * i));
        double rv[4] = {r0.x, r0.y, r1.x, r1.y}, uv[4] = {u0.x, u0.y, u1.x, u1.y};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double cj = (double)(float)cv[j], bj = (double)(float)bv[j];
            rv[j] = fmaT<double>(-cj, bj, rv[j]);
            uv[j] += cj;
        }
        st_nt<NTS>(r2, f64x2{rv[0], rv[1]});
        st_nt<NTS>(r2 + 1, f64x2{rv[2], rv[3]});
        st_nt<NTS>(u2, f64x2{uv[0], uv[1]});
        st_nt<NTS>(u2 + 1, f64x2{uv[2], uv[3]});
    }
}

static int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

static int stencil_chunks(int P, int zc) { return ceil_div(P - 1, zc); }

int stencil_blocks(int D, int P, const Shape &s) {
    if (D == 3 && s.ty > 0) return ceil_div(P - 1, s.ty) * stencil_chunks(P, s.zc);
    const long lines = (long)(D == 3 ? P : 1) * stencil_chunks(P, s.zc);
    return ceil_div((long)(P / s.V) * lines, s.bs);
}

template <class T> static int prec_of();
template <> int prec_of<double>() { return P_F64; }
template <> int prec_of<float>() { return P_F32; }
template <> int prec_of<f16>() { return P_F16; }
template <> int prec_of<bf16>() { return P_BF16; }

int restrict_blocks(int D, int P, const RShape &s) {
    const int Pc = P / 2;
    const int ytiles = D == 3 ? ceil_div(Pc - 1, s.tyc) : 1;
    return ytiles * ceil_div(Pc - 1, s.zcc);
}

size_t restrict_lds_bytes(int D, int P, int pf, const RShape &s) {
    const size_t acc = pf == P_F64 ? 8 : 4;
    if (D == 3 && s.pipe)
        return 2 * (size_t)(2 * s.tyc + 3) * P * prec_bytes(pf) +
               2 * (size_t)(2 * s.tyc + 1) * (s.pipe >= 2 ? P / 2 : P) * acc;
    const int G = D == 3 ? 2 * s.tyc + 1 : 1;
    return 2 * (size_t)G * P * acc;
}

int flat_blocks(long N) {
    long b = (N + 255) / 256;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

template <int D, int V, class F, class E>
static hipError_t run_stencil(const F &f, const E &e, int P, const Shape &s, hipStream_t st) {
    const int nch = stencil_chunks(P, s.zc);
    const int blocks = stencil_blocks(D, P, s);
    hipLaunchKernelGGL((k_stencil<D, V, F, E>), dim3(blocks), dim3(s.bs), 0, st, f, e, P, s.zc, nch, s.xcd);
    return hipGetLastError();
}

// Extra LDS of the staged prolongation field: three slots of z-interpolated
// coarse rows.
static size_t staged_ez_bytes(int P, int ty, size_t pa) { return 3 * (size_t)(ty / 2 + 3) * (P / 2 + 4) * pa; }

template <class F> struct StagedBytes {
    static size_t get(int P, int ty) { return 0; }
};
template <class TF, class TC, int V> struct StagedBytes<PProlS<TF, TC, V>> {
    static size_t get(int P, int ty) { return staged_ez_bytes(P, ty, sizeof(typename PProlS<TF, TC, V>::PA)); }
};

template <int V, class F, class E>
static hipError_t run_march(const F &f, const E &e, int P, const Shape &s, hipStream_t st) {
    const int ytiles = ceil_div(P - 1, s.ty);
    const int nch = stencil_chunks(P, s.zc);
    const int threads = (P / V) * (s.ty + 2);
    const size_t lds = march_lds_bytes(P, s.ty, sizeof(typename F::lds_t)) + StagedBytes<F>::get(P, s.ty);
    if (s.dp == 2 && !F::kStaged)
        hipLaunchKernelGGL((k_march<V, F, E, 2>), dim3(ytiles * nch), dim3(threads), lds, st, f, e, P, s.ty, s.zc,
                           ytiles, s.xcd);
    else
        hipLaunchKernelGGL((k_march<V, F, E, 1>), dim3(ytiles * nch), dim3(threads), lds, st, f, e, P, s.ty, s.zc,
                           ytiles, s.xcd);
    return hipGetLastError();
}

#define MG_DISPATCH_V(V, CALL)                        \
    do {                                              \
        if ((V) == 8) { constexpr int VV = 8; CALL; } \
        else { constexpr int VV = 4; CALL; }          \
    } while (0)

// Dispatch a (D, V) pair to a functor templated on them.
#define MG_DISPATCH_DV(D, V, CALL)                                   \
    do {                                                             \
        if ((D) == 3) {                                              \
            if ((V) == 8) { constexpr int DD = 3, VV = 8; CALL; }    \
            else { constexpr int DD = 3, VV = 4; CALL; }             \
        } else {                                                     \
            if ((V) == 8) { constexpr int DD = 2, VV = 8; CALL; }    \
            else { constexpr int DD = 2, VV = 4; CALL; }             \
        }                                                            \
    } while (0)

template <class T>
static hipError_t smooth_first_t(int D, int P, const void *b, const double *r, const double *scal, void *b_out,
                                 void *c, double omega, bool two, const Shape &s, hipStream_t st) {
    typedef acc_t<T> A;
    const A k = (A)(omega / (2.0 * D));
    T *cout = static_cast<T *>(c);
    hipError_t err = hipSuccess;
    if (D == 3 && s.ty > 0 && two) {
        if (r) {
            MG_DISPATCH_V(s.V, err = (run_march<VV>(PJac0Scaled<T, VV>{r, scal, k},
                                                   PSweep<T, VV, true, true>{nullptr, cout, static_cast<T *>(b_out), k},
                                                   P, s, st)));
        } else {
            MG_DISPATCH_V(s.V, err = (run_march<VV>(PJac0Arr<T, VV>{static_cast<const T *>(b), k},
                                                   PSweep<T, VV, true, false>{nullptr, cout, nullptr, k}, P, s, st)));
        }
        return err;
    }
    if (r) {
        typedef FScaled<T> R;
        typedef FJac0<T, R> F;
        const R rh{r, scal};
        const F f{rh, k};
        T *bo = static_cast<T *>(b_out);
        if (two) {
            const ESweep<T, R, true> e{rh, cout, bo, k};
            MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
        } else {
            const ECopy<T, R, true> e{rh, cout, bo};
            MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
        }
    } else {
        typedef FArr<T, A> R;
        typedef FJac0<T, R> F;
        const R rh{static_cast<const T *>(b)};
        const F f{rh, k};
        if (two) {
            const ESweep<T, R, false> e{rh, cout, nullptr, k};
            MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
        } else {
            const ECopy<T, R, false> e{rh, cout, nullptr};
            MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
        }
    }
    return err;
}

#define MG_DISPATCH_T(prec, CALL)                 \
    switch (prec) {                               \
    case P_F64: { typedef double TT; CALL; break; } \
    case P_F32: { typedef float TT; CALL; break; }  \
    case P_F16: { typedef f16 TT; CALL; break; }    \
    case P_BF16: { typedef bf16 TT; CALL; break; }  \
    default: return hipErrorInvalidValue;         \
    }

hipError_t launch_smooth_first(int D, int prec, int P, const void *b, const double *r, const double *scal,
                               void *b_out, void *c, double omega, bool two, const Shape &s, hipStream_t st) {
    MG_DISPATCH_T(prec, return smooth_first_t<TT>(D, P, b, r, scal, b_out, c, omega, two, s, st));
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t sweep_t(int D, int P, const void *b, const void *c, void *c_out, double omega, const Shape &s,
                          hipStream_t st) {
    typedef acc_t<T> A;
    typedef FArr<T, A> R;
    const R rh{static_cast<const T *>(b)};
    const R f{static_cast<const T *>(c)};
    const ESweep<T, R, false> e{rh, static_cast<T *>(c_out), nullptr, (A)(omega / (2.0 * D))};
    hipError_t err = hipSuccess;
    if (D == 3 && s.ty > 0) {
        MG_DISPATCH_V(s.V, err = (run_march<VV>(PArr<T, A, VV>{static_cast<const T *>(c)},
                                               PSweep<T, VV, false, false>{static_cast<const T *>(b),
                                                                           static_cast<T *>(c_out), nullptr,
                                                                           (A)(omega / (2.0 * D))},
                                               P, s, st)));
        return err;
    }
    MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
    return err;
}

hipError_t launch_sweep(int D, int prec, int P, const void *b, const void *c, void *c_out, double omega,
                        const Shape &s, hipStream_t st) {
    MG_DISPATCH_T(prec, return sweep_t<TT>(D, P, b, c, c_out, omega, s, st));
    return hipErrorInvalidValue;
}

template <class TF, class TC>
static hipError_t prolong_t(int D, int P, const void *c, const void *ec, const void *b, void *c_out, double omega,
                            bool sweep, const Shape &s, hipStream_t st) {
    typedef acc_t<TF> A;
    typedef FProl<TF, TC> F;
    typedef FArr<TF, A> R;
    const F f{static_cast<const TF *>(c), static_cast<const TC *>(ec), P / 2};
    const R rh{static_cast<const TF *>(b)};
    hipError_t err = hipSuccess;
    if (D == 3 && s.ty > 0 && sweep) {
        typedef typename FProl<TF, TC>::PA PA;
        const int nthr = (P / s.V) * (s.ty + 2);
        const bool staged = s.sg && P / 2 >= 8 &&
                            march_lds_bytes(P, s.ty, sizeof(TF)) + staged_ez_bytes(P, s.ty, sizeof(PA)) <= 65536 &&
                            (s.ty / 2 + 3) * (P / 2 + 4) <= 4 * nthr;
        if (staged) {
            MG_DISPATCH_V(s.V, err = (run_march<VV>(PProlS<TF, TC, VV>{static_cast<const TF *>(c),
                                                                       static_cast<const TC *>(ec), P / 2,
                                                                       nullptr, 0, 0, 0},
                                                   PSweep<TF, VV, false, false>{static_cast<const TF *>(b),
                                                                                static_cast<TF *>(c_out), nullptr,
                                                                                (A)(omega / (2.0 * D))},
                                                   P, s, st)));
            return err;
        }
        MG_DISPATCH_V(s.V, err = (run_march<VV>(PProl<TF, TC, VV>{static_cast<const TF *>(c),
                                                                  static_cast<const TC *>(ec), P / 2},
                                               PSweep<TF, VV, false, false>{static_cast<const TF *>(b),
                                                                            static_cast<TF *>(c_out), nullptr,
                                                                            (A)(omega / (2.0 * D))},
                                               P, s, st)));
        return err;
    }
    if (sweep) {
        const ESweep<TF, R, false> e{rh, static_cast<TF *>(c_out), nullptr, (A)(omega / (2.0 * D))};
        MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
    } else {
        const ECopy<TF, R, false> e{rh, static_cast<TF *>(c_out), nullptr};
        MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
    }
    return err;
}

template <class TF>
static hipError_t prolong_tf(int D, int pc, int P, const void *c, const void *ec, const void *b, void *c_out,
                             double omega, bool sweep, const Shape &s, hipStream_t st) {
    switch (pc) {
    case P_F64: return prolong_t<TF, double>(D, P, c, ec, b, c_out, omega, sweep, s, st);
    case P_F32: return prolong_t<TF, float>(D, P, c, ec, b, c_out, omega, sweep, s, st);
    case P_F16: return prolong_t<TF, f16>(D, P, c, ec, b, c_out, omega, sweep, s, st);
    case P_BF16: return prolong_t<TF, bf16>(D, P, c, ec, b, c_out, omega, sweep, s, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_prolong(int D, int pf, int pc, int P, const void *c, const void *ec, const void *b, void *c_out,
                          double omega, bool sweep, const Shape &s, hipStream_t st) {
    MG_DISPATCH_T(pf, return prolong_tf<TT>(D, pc, P, c, ec, b, c_out, omega, sweep, s, st));
    return hipErrorInvalidValue;
}

template <int D, int V, class TF, class TC>
static hipError_t restrict_run(int P, const void *b, const void *c, void *bc, const RShape &s, hipStream_t st) {
    const int Pc = P / 2;
    if (D == 3 && s.pipe) {
        const int ytiles = ceil_div(Pc - 1, s.tyc);
        const int blocks = ytiles * ceil_div(Pc - 1, s.zcc);
        const int threads = (2 * s.tyc + 3) * (P / V);
        const size_t lds = restrict_lds_bytes(D, P, prec_of<TF>(), s);
        if (s.pipe == 4)
            hipLaunchKernelGGL((k_restrict2<V, TF, TC, true, 3>), dim3(blocks), dim3(threads), lds, st,
                               static_cast<const TF *>(b), static_cast<const TF *>(c), static_cast<TC *>(bc), P,
                               s.tyc, s.zcc, ytiles, 1);
        else if (s.pipe == 3)
            hipLaunchKernelGGL((k_restrict2<V, TF, TC, true, 2>), dim3(blocks), dim3(threads), lds, st,
                               static_cast<const TF *>(b), static_cast<const TF *>(c), static_cast<TC *>(bc), P,
                               s.tyc, s.zcc, ytiles, 1);
        else if (s.pipe == 2)
            hipLaunchKernelGGL((k_restrict2<V, TF, TC, true>), dim3(blocks), dim3(threads), lds, st,
                               static_cast<const TF *>(b), static_cast<const TF *>(c), static_cast<TC *>(bc), P,
                               s.tyc, s.zcc, ytiles, 1);
        else
            hipLaunchKernelGGL((k_restrict2<V, TF, TC, false>), dim3(blocks), dim3(threads), lds, st,
                               static_cast<const TF *>(b), static_cast<const TF *>(c), static_cast<TC *>(bc), P,
                               s.tyc, s.zcc, ytiles, 1);
        return hipGetLastError();
    }
    const int ytiles = D == 3 ? ceil_div(Pc - 1, s.tyc) : 1;
    const int blocks = ytiles * ceil_div(Pc - 1, s.zcc);
    const int G = D == 3 ? 2 * s.tyc + 1 : 1;
    const int threads = G * (P / V);
    const size_t lds = 2 * (size_t)G * P * sizeof(acc_t<TF>);
    hipLaunchKernelGGL((k_restrict<D, V, TF, TC>), dim3(blocks), dim3(threads), lds, st,
                       static_cast<const TF *>(b), static_cast<const TF *>(c), static_cast<TC *>(bc), P, s.tyc,
                       s.zcc, ytiles);
    return hipGetLastError();
}

template <class TF, class TC>
static hipError_t restrict_t(int D, int P, const void *b, const void *c, void *bc, const RShape &s, hipStream_t st) {
    hipError_t err = hipSuccess;
    MG_DISPATCH_DV(D, s.V, err = (restrict_run<DD, VV, TF, TC>(P, b, c, bc, s, st)));
    return err;
}

template <class TF>
static hipError_t restrict_tf(int D, int pc, int P, const void *b, const void *c, void *bc, const RShape &s,
                              hipStream_t st) {
    switch (pc) {
    case P_F64: return restrict_t<TF, double>(D, P, b, c, bc, s, st);
    case P_F32: return restrict_t<TF, float>(D, P, b, c, bc, s, st);
    case P_F16: return restrict_t<TF, f16>(D, P, b, c, bc, s, st);
    case P_BF16: return restrict_t<TF, bf16>(D, P, b, c, bc, s, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_restrict(int D, int pf, int pc, int P, const void *b, const void *c, void *bc, const RShape &s,
                           hipStream_t st) {
    MG_DISPATCH_T(pf, return restrict_tf<TT>(D, pc, P, b, c, bc, s, st));
    return hipErrorInvalidValue;
}

hipError_t launch_coarse(int D, int prec, const void *b, void *c, hipStream_t st) {
    MG_DISPATCH_T(prec, {
        if (D == 3)
            hipLaunchKernelGGL((k_coarse<3, TT>), dim3(1), dim3(64), 0, st, static_cast<const TT *>(b),
                               static_cast<TT *>(c));
        else
            hipLaunchKernelGGL((k_coarse<2, TT>), dim3(1), dim3(64), 0, st, static_cast<const TT *>(b),
                               static_cast<TT *>(c));
        return hipGetLastError();
    });
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t outer_t(int D, int P, const void *c, double *R, double *U, const double *scal, double h2,
                          double *part, const Shape &s, hipStream_t st) {
    const FArr<T, double> f{static_cast<const T *>(c)};
    const EOuter e{R, U, scal, h2, part};
    hipError_t err = hipSuccess;
    if (D == 3 && s.ty > 0) {
        MG_DISPATCH_V(s.V, err = (run_march<VV>(PArr<T, double, VV>{static_cast<const T *>(c)},
                                               POuter<VV>{R, U, scal, h2, part}, P, s, st)));
        return err;
    }
    MG_DISPATCH_DV(D, s.V, err = (run_stencil<DD, VV>(f, e, P, s, st)));
    return err;
}

hipError_t launch_outer_update(int D, int prec, int P, const void *c, double *R, double *U, const double *scal,
                               double h2, double *part, const Shape &s, hipStream_t st) {
    MG_DISPATCH_T(prec, return outer_t<TT>(D, P, c, R, U, scal, h2, part, s, st));
    return hipErrorInvalidValue;
}

hipError_t launch_resid_flat(int D, int n, int P, const double *b, const double *U, double *R, double *uout,
                             double inv_h2, double *part, hipStream_t st) {
    const long N = D == 3 ? (long)n * n * n : (long)n * n;
    const int blocks = flat_blocks(N);
    if (D == 3) {
        // y bands of four rows; z chunks so that the tiles about fill the blocks
        const int ytiles = (n + 3) / 4;
        const int nzparts = std::max(1, (blocks + ytiles - 1) / ytiles);
        const int zc = std::max(1, (n + nzparts - 1) / nzparts);
        const int ntiles = ytiles * ((n + zc - 1) / zc);
        if (U) {
            // lane l holds x = l + 64 k, k < KX
            const int kx = (n + 63) / 64;
#define MG_RM(KX)                                                                                                  \
    hipLaunchKernelGGL(k_resid_march<KX>, dim3(blocks), dim3(256), 0, st, b, U, R, uout, n, P, inv_h2, part, ytiles, \
                       zc, ntiles)
            if (kx <= 1) MG_RM(1);
            else if (kx <= 2) MG_RM(2);
            else if (kx <= 4) MG_RM(4);
            else if (kx <= 8) MG_RM(8);
            else MG_RM(16);
#undef MG_RM
        } else {
            hipLaunchKernelGGL(k_resid_rows<3>, dim3(blocks), dim3(256), 0, st, b, U, R, uout, n, P, inv_h2, part);
        }
    } else
        hipLaunchKernelGGL(k_resid_rows<2>, dim3(blocks), dim3(256), 0, st, b, U, R, uout, n, P, inv_h2, part);
    return hipGetLastError();
}

hipError_t launch_defer_flush(int prec, const void *cdefer, size_t cstride, const double *adef, int count, double h2,
                              double *U, size_t elems, int *ctr, hipStream_t st, bool from_zero) {
    if (elems % 8 || count < 0) return hipErrorInvalidValue;
    const size_t n8 = elems / 8;
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>((n8 + 255) / 256, 8192));
#define MG_FL(T) \
    hipLaunchKernelGGL(k_defer_flush<T>, dim3(blocks), dim3(256), 0, st, static_cast<const T *>(cdefer), cstride, adef, \
                       count, h2, U, n8, ctr, from_zero ? 1 : 0)
    switch (prec) {
    case P_F64: MG_FL(double); break;
    case P_F32: MG_FL(float); break;
    case P_F16: MG_FL(f16); break;
    case P_BF16: MG_FL(bf16); break;
    default: return hipErrorInvalidValue;
    }
#undef MG_FL
    return hipGetLastError();
}

hipError_t launch_finalize(const double *part, int nparts, double *scal, int scaling, hipStream_t st, int *ctr) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, part, nparts, scal, scaling, ctr);
    return hipGetLastError();
}

template <class TS, class TD>
static hipError_t pack_t(int D, bool unpack, int n, int P, const void *src, void *dst, hipStream_t st) {
    const long N = D == 3 ? (long)n * n * n : (long)n * n;
    const int blocks = flat_blocks(N);
    const TS *s = static_cast<const TS *>(src);
    TD *d = static_cast<TD *>(dst);
    if (D == 3) {
        if (unpack) hipLaunchKernelGGL((k_unpack<3, TS, TD>), dim3(blocks), dim3(256), 0, st, s, d, n, P, N);
        else hipLaunchKernelGGL((k_pack<3, TS, TD>), dim3(blocks), dim3(256), 0, st, s, d, n, P, N);
    } else {
        if (unpack) hipLaunchKernelGGL((k_unpack<2, TS, TD>), dim3(blocks), dim3(256), 0, st, s, d, n, P, N);
        else hipLaunchKernelGGL((k_pack<2, TS, TD>), dim3(blocks), dim3(256), 0, st, s, d, n, P, N);
    }
    return hipGetLastError();
}

template <class TS>
static hipError_t pack_ts(int D, bool unpack, int dp, int n, int P, const void *src, void *dst, hipStream_t st) {
    switch (dp) {
    case P_F64: return pack_t<TS, double>(D, unpack, n, P, src, dst, st);
    case P_F32: return pack_t<TS, float>(D, unpack, n, P, src, dst, st);
    case P_F16: return pack_t<TS, f16>(D, unpack, n, P, src, dst, st);
    case P_BF16: return pack_t<TS, bf16>(D, unpack, n, P, src, dst, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pack(int D, int sp, int dp, int n, int P, const void *src, void *dst, hipStream_t st) {
    MG_DISPATCH_T(sp, return pack_ts<TT>(D, false, dp, n, P, src, dst, st));
    return hipErrorInvalidValue;
}

hipError_t launch_unpack(int D, int sp, int dp, int n, int P, const void *src, void *dst, hipStream_t st) {
    MG_DISPATCH_T(sp, return pack_ts<TT>(D, true, dp, n, P, src, dst, st));
    return hipErrorInvalidValue;
}

hipError_t launch_probe(void *dst, const void *src, size_t bytes, int kind, int blocks, unsigned *sink,
                        hipStream_t st) {
    if (bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
        return hipErrorInvalidValue;
    if (kind == 3 || kind == 6 || kind == 7) {
        // dst: R and U, bytes each; src: c and b, bytes / 4 each (FP16)
        if (bytes % 32) return hipErrorInvalidValue;
        double *R = static_cast<double *>(dst);
        const f16 *c = static_cast<const f16 *>(src);
        if (kind == 3)
            hipLaunchKernelGGL((k_probe_update<false, false>), dim3((unsigned)blocks), dim3(256), 0, st, R,
                               R + bytes / 8, c, c + bytes / 8, bytes / 32);
        else if (kind == 6)
            hipLaunchKernelGGL((k_probe_update<true, true>), dim3((unsigned)blocks), dim3(256), 0, st, R,
                               R + bytes / 8, c, c + bytes / 8, bytes / 32);
        else
            hipLaunchKernelGGL((k_probe_update<false, true>), dim3((unsigned)blocks), dim3(256), 0, st, R,
                               R + bytes / 8, c, c + bytes / 8, bytes / 32);
        return hipGetLastError();
    }
    if (kind < 0 || kind > 5) return hipErrorInvalidValue;
    if (kind >= 3)
        hipLaunchKernelGGL(k_probe<true>, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<u32x4 *>(dst),
                           static_cast<const u32x4 *>(src), bytes / 16, kind - 3, sink);
    else
        hipLaunchKernelGGL(k_probe<false>, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<u32x4 *>(dst),
                           static_cast<const u32x4 *>(src), bytes / 16, kind, sink);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes % 16 || reinterpret_cast<uintptr_t>(p) % 16) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    long b = (long)((n16 + 255) / 256);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)b), dim3(256), 0, st, static_cast<uint4 *>(p), n16);
    return hipGetLastError();
}

}  // namespace mg

// ===========================================================================
// Batched instances: one persistent launch per V-cycle stage walks a work list
// of (descriptor, tile) items that spans all instances whose grids have that
// stage; the per-tile work is the same device code as the single-grid
// kernels, so a batched instance computes exactly what it would alone.
// Instances whose device flag active[inst] is 0 are skipped (converged).
// ===========================================================================
namespace mg {

template <int V, int KIND, class T, class TC>
__global__ __launch_bounds__(256) void k_batched_stencil(const BDesc *__restrict__ descs,
                                                         const BItem *__restrict__ items, int nitems,
                                                         const int *__restrict__ active, double omega,
                                                         double *__restrict__ part) {
    __shared__ double red[8];
    typedef acc_t<T> A;
    const A k = (A)(omega / 6.0);
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem item = items[it];
        const BDesc &d = descs[item.d];
        if (!active[d.inst]) continue;
        if constexpr (KIND == BK_SMOOTH2) {
            typedef FArr<T, A> R;
            const R rh{static_cast<const T *>(d.b)};
            const FJac0<T, R> f{rh, k};
            const ESweep<T, R, false> e{rh, static_cast<T *>(d.cout), nullptr, k};
            stencil_body<3, V>(f, e, d.P, d.zc, d.nchunks, item.blk, red, 0);
        } else if constexpr (KIND == BK_SMOOTH2_SCALED) {
            typedef FScaled<T> R;
            const R rh{static_cast<const double *>(d.b), d.scal};
            const FJac0<T, R> f{rh, k};
            const ESweep<T, R, true> e{rh, static_cast<T *>(d.cout), static_cast<T *>(d.bout), k};
            stencil_body<3, V>(f, e, d.P, d.zc, d.nchunks, item.blk, red, 0);
        } else if constexpr (KIND == BK_SWEEP) {
            typedef FArr<T, A> R;
            const R f{static_cast<const T *>(d.cin)};
            const ESweep<T, R, false> e{R{static_cast<const T *>(d.b)}, static_cast<T *>(d.cout), nullptr, k};
            stencil_body<3, V>(f, e, d.P, d.zc, d.nchunks, item.blk, red, 0);
        } else if constexpr (KIND == BK_PROLONG) {
            typedef FArr<T, A> R;
            const FProl<T, TC> f{static_cast<const T *>(d.cin), static_cast<const TC *>(d.ec), d.P / 2};
            const ESweep<T, R, false> e{R{static_cast<const T *>(d.b)}, static_cast<T *>(d.cout), nullptr, k};
            stencil_body<3, V>(f, e, d.P, d.zc, d.nchunks, item.blk, red, 0);
        } else {
            const FArr<T, double> f{static_cast<const T *>(d.cin)};
            const EOuter e{d.R, d.U, d.scal, d.h2, part};
            stencil_body<3, V>(f, e, d.P, d.zc, d.nchunks, item.blk, red, (long)d.part_off + item.blk);
        }
    }
}

template <int V, class TF, class TC>
__global__ __launch_bounds__(1024) void k_batched_restrict(const BDesc *__restrict__ descs,
                                                           const BItem *__restrict__ items, int nitems,
                                                           const int *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem item = items[it];
        const BDesc &d = descs[item.d];
        if (!active[d.inst]) continue;
        restrict_body<3, V, TF, TC>(static_cast<const TF *>(d.b), static_cast<const TF *>(d.cin),
                                    static_cast<TC *>(d.cout), d.P, d.tyc, d.zcc, d.ytiles, item.blk, smem_raw);
        __syncthreads();  // the next item reuses the LDS rows
    }
}

template <class T>
__global__ void k_batched_coarse(const BDesc *__restrict__ descs, int n, const int *__restrict__ active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !active[descs[i].inst]) return;
    typedef acc_t<T> A;
    const T *b = static_cast<const T *>(descs[i].b);
    T *c = static_cast<T *>(descs[i].cout);
    c[7] = Store<T>::from_acc(widen(b[7]) / A(6));
}

// One block per instance: reduce its partials into its scalars.
__global__ __launch_bounds__(256) void k_batched_finalize(const BFin *__restrict__ fin,
                                                          const int *__restrict__ active) {
    __shared__ double red[8];
    if (!active[blockIdx.x]) return;
    const BFin f = fin[blockIdx.x];
    double s = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < f.count; i += blockDim.x) {
        s += f.part[2 * i];
        m = nanmax(m, f.part[2 * i + 1]);
    }
    block_reduce(s, m, red);
    if (threadIdx.x == 0) {
        double a = f.ascale ? ldexp(m, f.ascale - 1) : 1.0;
        if (!(a > 0.0) || a > 1.7e308) a = 1.0;
        f.scal[0] = a;
        f.scal[1] = 1.0 / a;
        f.scal[2] = sqrt(s);
        f.scal[3] = m;
    }
}

// LDS-plane forms: the same per-tile bodies as k_march and k_restrict2.
template <int V, int KIND, class T, class TC>
__global__ __launch_bounds__(1024) void k_batched_march(const BDesc *__restrict__ descs,
                                                        const BItem *__restrict__ items, int nitems,
                                                        const int *__restrict__ active, double omega,
                                                        double *__restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[32];
    typedef acc_t<T> A;
    const A k = (A)(omega / 6.0);
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem item = items[it];
        const BDesc &d = descs[item.d];
        if (!active[d.inst]) continue;
        if constexpr (KIND == BK_SMOOTH2) {
            typedef PJac0Arr<T, V> F;
            typedef PSweep<T, V, true, false> E;
            march_body<V, F, E, 1>(F{static_cast<const T *>(d.b), k}, E{nullptr, static_cast<T *>(d.cout), nullptr, k},
                                   d.P, d.ty, d.zc, d.ytiles, item.blk, 0, smem_raw, red);
        } else if constexpr (KIND == BK_SMOOTH2_SCALED) {
            typedef PJac0Scaled<T, V> F;
            typedef PSweep<T, V, true, true> E;
            march_body<V, F, E, 1>(F{static_cast<const double *>(d.b), d.scal, k},
                                   E{nullptr, static_cast<T *>(d.cout), static_cast<T *>(d.bout), k}, d.P, d.ty,
                                   d.zc, d.ytiles, item.blk, 0, smem_raw, red);
        } else if constexpr (KIND == BK_SWEEP) {
            typedef PArr<T, A, V> F;
            typedef PSweep<T, V, false, false> E;
            march_body<V, F, E, 1>(F{static_cast<const T *>(d.cin)},
                                   E{static_cast<const T *>(d.b), static_cast<T *>(d.cout), nullptr, k}, d.P, d.ty,
                                   d.zc, d.ytiles, item.blk, 0, smem_raw, red);
        } else if constexpr (KIND == BK_PROLONG) {
            typedef PProl<T, TC, V> F;
            typedef PSweep<T, V, false, false> E;
            march_body<V, F, E, 1>(F{static_cast<const T *>(d.cin), static_cast<const TC *>(d.ec), d.P / 2},
                                   E{static_cast<const T *>(d.b), static_cast<T *>(d.cout), nullptr, k}, d.P, d.ty,
                                   d.zc, d.ytiles, item.blk, 0, smem_raw, red);
        } else {
            typedef PArr<T, double, V> F;
            typedef POuter<V> E;
            march_body<V, F, E, 1>(F{static_cast<const T *>(d.cin)}, E{d.R, d.U, d.scal, d.h2, part}, d.P, d.ty, d.zc,
                                   d.ytiles, item.blk, (long)d.part_off + item.blk, smem_raw, red);
        }
        __syncthreads();  // the next item reuses the LDS slots
    }
}

template <int V, class TF, class TC, bool XSH>
__global__ __launch_bounds__(1024) void k_batched_restrict2(const BDesc *__restrict__ descs,
                                                            const BItem *__restrict__ items, int nitems,
                                                            const int *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem item = items[it];
        const BDesc &d = descs[item.d];
        if (!active[d.inst]) continue;
        restrict2_body<V, TF, TC, XSH, XSH ? 2 : 1>(static_cast<const TF *>(d.b), static_cast<const TF *>(d.cin),
                                                    static_cast<TC *>(d.cout), d.P, d.tyc, d.zcc, d.ytiles, item.blk,
                                                    smem_raw);
        __syncthreads();
    }
}

#define MG_BT(prec, ...)                                   \
    switch (prec) {                                        \
    case P_F64: { typedef double TB; __VA_ARGS__; break; } \
    case P_F32: { typedef float TB; __VA_ARGS__; break; }  \
    case P_F16: { typedef f16 TB; __VA_ARGS__; break; }    \
    case P_BF16: { typedef bf16 TB; __VA_ARGS__; break; }  \
    default: return hipErrorInvalidValue;                  \
    }

template <int V, int KIND, class T>
static hipError_t bst_tc(int pc, const BDesc *d, const BItem *it, int n, const int *act, double omega, double *part,
                         int grid, hipStream_t st) {
    switch (pc) {
    case P_F64:
        hipLaunchKernelGGL((k_batched_stencil<V, KIND, T, double>), dim3(grid), dim3(256), 0, st, d, it, n, act,
                           omega, part);
        break;
    case P_F32:
        hipLaunchKernelGGL((k_batched_stencil<V, KIND, T, float>), dim3(grid), dim3(256), 0, st, d, it, n, act,
                           omega, part);
        break;
    case P_F16:
        hipLaunchKernelGGL((k_batched_stencil<V, KIND, T, f16>), dim3(grid), dim3(256), 0, st, d, it, n, act,
                           omega, part);
        break;
    case P_BF16:
        hipLaunchKernelGGL((k_batched_stencil<V, KIND, T, bf16>), dim3(grid), dim3(256), 0, st, d, it, n, act,
                           omega, part);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND>
static hipError_t bst_kind(int V, int pf, int pc, const BDesc *d, const BItem *it, int n, const int *act,
                           double omega, double *part, int grid, hipStream_t st) {
    if (KIND != BK_PROLONG) pc = P_F64;  // the coarse format only matters for prolongation
    MG_BT(pf, {
        if (V == 8) return bst_tc<8, KIND, TB>(pc, d, it, n, act, omega, part, grid, st);
        return bst_tc<4, KIND, TB>(pc, d, it, n, act, omega, part, grid, st);
    });
    return hipErrorInvalidValue;
}

hipError_t launch_batched_stencil(int kind, int V, int pf, int pc, const BDesc *d, const BItem *items, int nitems,
                                  const int *active, double omega, double *part, int grid, hipStream_t st) {
    switch (kind) {
    case BK_SMOOTH2: return bst_kind<BK_SMOOTH2>(V, pf, pc, d, items, nitems, active, omega, part, grid, st);
    case BK_SMOOTH2_SCALED:
        return bst_kind<BK_SMOOTH2_SCALED>(V, pf, pc, d, items, nitems, active, omega, part, grid, st);
    case BK_SWEEP: return bst_kind<BK_SWEEP>(V, pf, pc, d, items, nitems, active, omega, part, grid, st);
    case BK_PROLONG: return bst_kind<BK_PROLONG>(V, pf, pc, d, items, nitems, active, omega, part, grid, st);
    case BK_OUTER: return bst_kind<BK_OUTER>(V, pf, pc, d, items, nitems, active, omega, part, grid, st);
    }
    return hipErrorInvalidValue;
}

template <int V, class TF>
static hipError_t brs_tc(int pc, const BDesc *d, const BItem *it, int n, const int *act, int grid, int threads,
                         size_t lds, hipStream_t st) {
    switch (pc) {
    case P_F64:
        hipLaunchKernelGGL((k_batched_restrict<V, TF, double>), dim3(grid), dim3(threads), lds, st, d, it, n, act);
        break;
    case P_F32:
        hipLaunchKernelGGL((k_batched_restrict<V, TF, float>), dim3(grid), dim3(threads), lds, st, d, it, n, act);
        break;
    case P_F16:
        hipLaunchKernelGGL((k_batched_restrict<V, TF, f16>), dim3(grid), dim3(threads), lds, st, d, it, n, act);
        break;
    case P_BF16:
        hipLaunchKernelGGL((k_batched_restrict<V, TF, bf16>), dim3(grid), dim3(threads), lds, st, d, it, n, act);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batched_restrict(int V, int pf, int pc, const BDesc *d, const BItem *items, int nitems,
                                   const int *active, int grid, int threads, size_t lds, hipStream_t st) {
    MG_BT(pf, {
        if (V == 8) return brs_tc<8, TB>(pc, d, items, nitems, active, grid, threads, lds, st);
        return brs_tc<4, TB>(pc, d, items, nitems, active, grid, threads, lds, st);
    });
    return hipErrorInvalidValue;
}

hipError_t launch_batched_coarse(int prec, const BDesc *d, int n, const int *active, hipStream_t st) {
    const int grid = (n + 63) / 64;
    MG_BT(prec, {
        hipLaunchKernelGGL((k_batched_coarse<TB>), dim3(grid), dim3(64), 0, st, d, n, active);
        return hipGetLastError();
    });
    return hipErrorInvalidValue;
}

template <int KIND, class T, int V>
static hipError_t bmarch_tc(int pc, const BDesc *d, const BItem *it, int n, const int *act, double omega,
                            double *part, int grid, int threads, size_t lds, hipStream_t st) {
    if constexpr (KIND == BK_PROLONG) {
        MG_BT(pc, hipLaunchKernelGGL((k_batched_march<V, KIND, T, TB>), dim3(grid), dim3(threads), lds, st, d, it, n,
                                     act, omega, part));
    } else {
        hipLaunchKernelGGL((k_batched_march<V, KIND, T, double>), dim3(grid), dim3(threads), lds, st, d, it, n, act,
                           omega, part);
    }
    return hipGetLastError();
}

template <int KIND>
static hipError_t bmarch_kind(int V, int pf, int pc, const BDesc *d, const BItem *it, int n, const int *act,
                              double omega, double *part, int grid, int threads, size_t lds, hipStream_t st) {
    // FP64 rows and the FP64 update use V = 4 (V = 8 spills registers)
    if (V != 4 && V != 8) return hipErrorInvalidValue;
    if constexpr (KIND == BK_OUTER) {
        if (V != 4) return hipErrorInvalidValue;
        MG_BT(pf, return (bmarch_tc<KIND, TB, 4>(pc, d, it, n, act, omega, part, grid, threads, lds, st)));
    } else {
        if (pf == P_F64) {
            if (V != 4) return hipErrorInvalidValue;
            return bmarch_tc<KIND, double, 4>(pc, d, it, n, act, omega, part, grid, threads, lds, st);
        }
        switch (pf) {
        case P_F32:
            return V == 8 ? bmarch_tc<KIND, float, 8>(pc, d, it, n, act, omega, part, grid, threads, lds, st)
                          : bmarch_tc<KIND, float, 4>(pc, d, it, n, act, omega, part, grid, threads, lds, st);
        case P_F16:
            return V == 8 ? bmarch_tc<KIND, f16, 8>(pc, d, it, n, act, omega, part, grid, threads, lds, st)
                          : bmarch_tc<KIND, f16, 4>(pc, d, it, n, act, omega, part, grid, threads, lds, st);
        case P_BF16:
            return V == 8 ? bmarch_tc<KIND, bf16, 8>(pc, d, it, n, act, omega, part, grid, threads, lds, st)
                          : bmarch_tc<KIND, bf16, 4>(pc, d, it, n, act, omega, part, grid, threads, lds, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batched_march(int kind, int V, int pf, int pc, const BDesc *d, const BItem *items, int nitems,
                                const int *active, double omega, double *part, int grid, int threads, size_t lds,
                                hipStream_t st) {
    switch (kind) {
    case BK_SMOOTH2:
        return bmarch_kind<BK_SMOOTH2>(V, pf, pc, d, items, nitems, active, omega, part, grid, threads, lds, st);
    case BK_SMOOTH2_SCALED:
        return bmarch_kind<BK_SMOOTH2_SCALED>(V, pf, pc, d, items, nitems, active, omega, part, grid, threads, lds,
                                              st);
    case BK_SWEEP:
        return bmarch_kind<BK_SWEEP>(V, pf, pc, d, items, nitems, active, omega, part, grid, threads, lds, st);
    case BK_PROLONG:
        return bmarch_kind<BK_PROLONG>(V, pf, pc, d, items, nitems, active, omega, part, grid, threads, lds, st);
    case BK_OUTER:
        return bmarch_kind<BK_OUTER>(V, pf, pc, d, items, nitems, active, omega, part, grid, threads, lds, st);
    }
    return hipErrorInvalidValue;
}

template <int V, class TF, bool XSH>
static hipError_t brs2_tc(int pc, const BDesc *d, const BItem *it, int n, const int *act, int grid, int threads,
                          size_t lds, hipStream_t st) {
    MG_BT(pc, hipLaunchKernelGGL((k_batched_restrict2<V, TF, TB, XSH>), dim3(grid), dim3(threads), lds, st, d, it, n,
                                 act));
    return hipGetLastError();
}

hipError_t launch_batched_restrict2(int V, int pf, int pc, bool xsh, const BDesc *d, const BItem *items, int nitems,
                                    const int *active, int grid, int threads, size_t lds, hipStream_t st) {
    if (pf == P_F64) {
        if (V != 4) return hipErrorInvalidValue;
        return xsh ? brs2_tc<4, double, true>(pc, d, items, nitems, active, grid, threads, lds, st)
                   : brs2_tc<4, double, false>(pc, d, items, nitems, active, grid, threads, lds, st);
    }
    switch (pf) {
    case P_F32:
        if (V == 8) return xsh ? brs2_tc<8, float, true>(pc, d, items, nitems, active, grid, threads, lds, st)
                               : brs2_tc<8, float, false>(pc, d, items, nitems, active, grid, threads, lds, st);
        return xsh ? brs2_tc<4, float, true>(pc, d, items, nitems, active, grid, threads, lds, st)
                   : brs2_tc<4, float, false>(pc, d, items, nitems, active, grid, threads, lds, st);
    case P_F16:
        if (V == 8) return xsh ? brs2_tc<8, f16, true>(pc, d, items, nitems, active, grid, threads, lds, st)
                               : brs2_tc<8, f16, false>(pc, d, items, nitems, active, grid, threads, lds, st);
        return xsh ? brs2_tc<4, f16, true>(pc, d, items, nitems, active, grid, threads, lds, st)
                   : brs2_tc<4, f16, false>(pc, d, items, nitems, active, grid, threads, lds, st);
    case P_BF16:
        if (V == 8) return xsh ? brs2_tc<8, bf16, true>(pc, d, items, nitems, active, grid, threads, lds, st)
                               : brs2_tc<8, bf16, false>(pc, d, items, nitems, active, grid, threads, lds, st);
        return xsh ? brs2_tc<4, bf16, true>(pc, d, items, nitems, active, grid, threads, lds, st)
                   : brs2_tc<4, bf16, false>(pc, d, items, nitems, active, grid, threads, lds, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batched_finalize(const BFin *fin, int ninst, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(k_batched_finalize, dim3(ninst), dim3(256), 0, st, fin, active);
    return hipGetLastError();
}

}  // namespace mg
