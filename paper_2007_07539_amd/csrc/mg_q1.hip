// The V-cycle and refinement kernels for the Q1 finite-element discretisation
// that the paper's measurements use (Section 5: bilinear elements on the unit
// square, trilinear on the unit cube).
//
// Units.  With the grid-scaled correction c = h^(D-2) e on every level, the
// level operator h^(D-2) S becomes the constant stencil S (q1_weighted), the
// restriction is full weighting (weights (1/4, 1/2, 1/4) per axis, summing to
// one: the finite-element restriction P^T divided by 2^D) and the
// prolongation carries a factor 4, exactly as for the finite-difference
// operator: P^T A_h P = A_2h for Q1, and (A_h = h^(D-2) S) the coarse
// correction equation S c_2h = FW r_h then reproduces the physical two-grid
// correction.  Magnitudes stay level-independent, which half precision needs.
//
// Damped Jacobi: c <- c + omega (b - S c) / diag(S), diag(S) = 8/3 in 2-D and
// 3-D.  Arithmetic in the level's accumulator format (FP32 for FP32, FP16 and
// BF16 storage, FP64 for FP64), one rounding into the storage format per
// stored value.  The kernels read neighbours through the caches, consecutive
// threads on consecutive x.  Where the pitch is a multiple of 4 the sweep, the
// residual and the FP64 update take four x points per thread with one vector
// load per row: in 3-D marching z with three planes of row sums kept in
// registers, in 2-D row by row.  On 3-D levels stored in a 2-byte format they
// run as one LDS-staged kernel (k_q1_lds: a block's rows and the two around
// them staged plane by plane, so each plane is read once per block row), which
// also fuses the residual with its restriction and forms the final FP64 check
// b - S u.  Elsewhere they take one point per thread on a (x blocks, n, n)
// grid.  The first sweep from zero and the interpolation take four fine points
// per thread (each coarse value loaded once).  The restriction and
// interpolation remap work-group numbers so that each XCD takes one contiguous
// range of points.
#include "mg_device.h"
#include "mg_launch.h"

namespace mg {
namespace {

constexpr int kThreads = 256;

// Interior point number i (x fastest) -> padded offset.
template <int D> __device__ __forceinline__ size_t q1_at(unsigned i, int n, int P, int &x, int &y, int &z) {
    x = (int)(i % (unsigned)n) + 1;
    const unsigned rest = i / (unsigned)n;
    if (D == 3) {
        y = (int)(rest % (unsigned)n) + 1;
        z = (int)(rest / (unsigned)n) + 1;
    } else {
        y = 0;
        z = (int)rest + 1;
    }
    return Grid<D>{P}.at(x, y, z);
}

// Point of a (x blocks, n, n) grid (3-D) or (x blocks, n) grid (2-D): no
// division; false beyond the row.
template <int D> __device__ __forceinline__ bool q1_point(int n, int P, size_t &o) {
    const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x) + 1;
    if (x > n) return false;
    o = D == 3 ? Grid<3>{P}.at(x, (int)blockIdx.y + 1, (int)blockIdx.z + 1) : Grid<2>{P}.at(x, 0, (int)blockIdx.y + 1);
    return true;
}

__device__ __forceinline__ unsigned q1_index(int xcd) {
    const int b = xcd ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    return (unsigned)b * kThreads + threadIdx.x;
}

// Row segments of kV points for the interpolation: segment t covers x0 ..
// x0 + kV - 1 of one row (points beyond n are not stored).
constexpr int kV = 4;
__host__ __device__ __forceinline__ unsigned q1_segs_per_row(int n) { return (unsigned)(n + kV - 1) / kV; }
__host__ __device__ __forceinline__ unsigned q1_segs(int D, int n) {
    return q1_segs_per_row(n) * (D == 3 ? (unsigned)n * n : (unsigned)n);
}

// First Jacobi iterate from c = 0: c = round(w b), w = omega / diag(S).
// FROM_R: the right-hand side is the FP64 residual times 1/alpha (scal[1]),
// rounded once into the level format and stored as b-hat as well.
template <int D, class T, bool FROM_R>
__global__ __launch_bounds__(kThreads) void k_q1_first(const T *__restrict__ b, const double *__restrict__ R,
                                                       const double *__restrict__ scal, T *__restrict__ bout,
                                                       T *__restrict__ cout, int n, int P, acc_t<T> w) {
    typedef acc_t<T> A;
    size_t o;
    if (!q1_point<D>(n, P, o)) return;
    A bv;
    if (FROM_R) {
        const T bh = Store<T>::from_f64(R[o] * scal[1]);
        bout[o] = bh;
        bv = (A)widen(bh);
    } else {
        bv = (A)widen(b[o]);
    }
    cout[o] = Store<T>::from_acc(w * bv);
}

// The same first sweep on a pitch that is a multiple of 4: one thread per
// four-point segment x0 = 4t of a row (vector loads and stores; the ghost
// x = 0 of the first segment receives zero, as it holds).
template <int D, class T, bool FROM_R>
__global__ __launch_bounds__(kThreads) void k_q1_first4(const T *__restrict__ b, const double *__restrict__ R,
                                                        const double *__restrict__ scal, T *__restrict__ bout,
                                                        T *__restrict__ cout, int n, int P, acc_t<T> w) {
    typedef acc_t<T> A;
    const int TX = P / 4;
    const long rows = D == 3 ? (long)n * n : (long)n;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)TX * rows) return;
    const int tx = (int)(t % TX);
    const long row = t / TX;
    const int y = D == 3 ? (int)(row % n) + 1 : 0;
    const int z = D == 3 ? (int)(row / n) + 1 : (int)row + 1;
    const size_t o = Grid<D>{P}.at(4 * tx, y, z);
    A bv[4];
    if constexpr (FROM_R) {
        double rv[4];
        load_row<double, 4>(R + o, rv);
        const double inv = scal[1];
        T bh[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) bh[i] = Store<T>::from_f64(rv[i] * inv);
        if (tx == 0) bh[0] = zero_of<T>();
        store_row<T, 4>(bout + o, bh);
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = (A)widen(bh[i]);
    } else {
        load_row<T, 4>(b + o, bv);
        if (tx == 0) bv[0] = A(0);
    }
    T cv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) cv[i] = Store<T>::from_acc(w * bv[i]);
    store_row<T, 4>(cout + o, cv);
}

// One Jacobi sweep: cout = c + w (b - S c).
template <int D, class T>
__global__ __launch_bounds__(kThreads) void k_q1_sweep(const T *__restrict__ b, const T *__restrict__ c,
                                                       T *__restrict__ cout, int n, int P, acc_t<T> w) {
    typedef acc_t<T> A;
    size_t o;
    if (!q1_point<D>(n, P, o)) return;
    const A sc = q1_weighted<D, A>(c, o, P) * q1_scale<D, A>();
    const A r = (A)widen(b[o]) - sc;
    cout[o] = Store<T>::from_acc(fmaT<A>(w, r, (A)widen(c[o])));
}

// Fine residual r = b - S c in the accumulator format (the restriction's input).
template <int D, class T>
__global__ __launch_bounds__(kThreads) void k_q1_resid(const T *__restrict__ b, const T *__restrict__ c,
                                                       acc_t<T> *__restrict__ r, int n, int P) {
    typedef acc_t<T> A;
    size_t o;
    if (!q1_point<D>(n, P, o)) return;
    r[o] = (A)widen(b[o]) - q1_weighted<D, A>(c, o, P) * q1_scale<D, A>();
}

// Four-point forms for levels whose pitch P is a multiple of 4 (2-D here; 3-D
// below, marching z): a thread takes
// x = 4j .. 4j+3 of one row (x = 0 is the ghost and is not stored), so every
// row segment starts on a 4-element boundary and is read with one vector load;
// x - 1 and x + 4 are single loads (for j = 0, x - 1 only serves the ghost and
// the ghost itself is read in its place).  Grid (P/4 / threads, n).
template <class T, class A> __device__ __forceinline__ void q1_load4(const T *p, A (&o)[4]) {
    T v[4];
    __builtin_memcpy(v, __builtin_assume_aligned(p, 4 * sizeof(T)), sizeof(v));
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = (A)widen(v[i]);
}

// w[k], k = 0..5: the row at x0 - 1 .. x0 + 4
template <class T, class A> __device__ __forceinline__ void q1_row6(const T *r, bool first, A (&w)[6]) {
    A m[4];
    q1_load4<T, A>(r, m);
    w[0] = (A)widen(r[first ? 0 : -1]);  // first: the ghost x = 0 itself (zero), never x = -1
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i + 1] = m[i];
    w[5] = (A)widen(r[4]);
}

template <int D> __device__ __forceinline__ bool q1_seg4(int P, size_t &o, int &x0) {
    x0 = 4 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (x0 >= P) return false;
    o = D == 3 ? Grid<3>{P}.at(x0, (int)blockIdx.y + 1, (int)blockIdx.z + 1) : Grid<2>{P}.at(x0, 0, (int)blockIdx.y + 1);
    return true;
}

// t[i] = 3 S v at x0 + i, 2-D (same weights as q1_weighted; the 3-D levels
// use the marching kernels below)
template <int D, class A, class T>
__device__ __forceinline__ void q1_weighted4(const T *__restrict__ v, size_t o, int P, bool first, A (&t)[4]) {
    static_assert(D == 2, "the 3-D four-point forms march z (k_q1_march4)");
    const T *c = v + o;
    const long Y = P;
    A cc[6], s[6], n[6];
    q1_row6<T, A>(c, first, cc);
    q1_row6<T, A>(c - Y, first, s);
    q1_row6<T, A>(c + Y, first, n);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const A nb = ((s[i] + s[i + 1]) + (s[i + 2] + cc[i])) + ((cc[i + 2] + n[i]) + (n[i + 1] + n[i + 2]));
        t[i] = fmaT<A>(A(8), cc[i + 1], -nb);
    }
}

template <int D, class T>
__global__ __launch_bounds__(kThreads) void k_q1_sweep4(const T *__restrict__ b, const T *__restrict__ c,
                                                        T *__restrict__ cout, int P, acc_t<T> w) {
    typedef acc_t<T> A;
    size_t o;
    int x0;
    if (!q1_seg4<D>(P, o, x0)) return;
    A s[4], bv[4], cv[4];
    q1_weighted4<D, A>(c, o, P, x0 == 0, s);
    q1_load4<T, A>(b + o, bv);
    q1_load4<T, A>(c + o, cv);
    T ov[4];  // x = 0 (first segment) is the ghost and receives zero
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const A r = bv[i] - s[i] * q1_scale<D, A>();
        ov[i] = (i == 0 && x0 == 0) ? zero_of<T>() : Store<T>::from_acc(fmaT<A>(w, r, cv[i]));
    }
    store_row<T, 4>(cout + o, ov);
}

template <int D, class T>
__global__ __launch_bounds__(kThreads) void k_q1_resid4(const T *__restrict__ b, const T *__restrict__ c,
                                                        acc_t<T> *__restrict__ r, int P) {
    typedef acc_t<T> A;
    size_t o;
    int x0;
    if (!q1_seg4<D>(P, o, x0)) return;
    A s[4], bv[4];
    q1_weighted4<D, A>(c, o, P, x0 == 0, s);
    q1_load4<T, A>(b + o, bv);
    A ov[4];  // x = 0 (first segment) is the ghost and receives zero
#pragma unroll
    for (int i = 0; i < 4; ++i) ov[i] = (i == 0 && x0 == 0) ? A(0) : bv[i] - s[i] * q1_scale<D, A>();
    store_row<A, 4>(r + o, ov);
}

// The three rows y, y - 1, y + 1 of one plane that a four-point segment needs
// (x0 - 1 .. x0 + 4), still in the storage format: loaded one plane ahead of
// their use by the marching kernels.
template <class T> struct Q1Plane {
    RawRow<T, 4> m[3];  // x0 .. x0 + 3 of rows y, y - 1, y + 1
    T l[3], r[3];       // x0 - 1 (the ghost x = 0 itself for the first segment) and x0 + 4
};
template <class T>
__device__ __forceinline__ void q1_fetch_plane(const T *row, long Y, bool first, Q1Plane<T> &p) {
    const T *rows[3] = {row, row - Y, row + Y};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fetch_row<T, 4>(rows[k], p.m[k]);
        p.l[k] = rows[k][first ? 0 : -1];
        p.r[k] = rows[k][4];
    }
}
// C = row y and A = row (y - 1) + row (y + 1), as q1_row6 forms them
template <class T, class A>
__device__ __forceinline__ void q1_widen_plane(const Q1Plane<T> &p, A (&Av)[6], A (&Cv)[6]) {
    A w[3][6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        A m[4];
        widen_row<T, 4>(p.m[k], m);
        w[k][0] = (A)widen(p.l[k]);
#pragma unroll
        for (int i = 0; i < 4; ++i) w[k][i + 1] = m[i];
        w[k][5] = (A)widen(p.r[k]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        Cv[k] = w[0][k];
        Av[k] = w[1][k] + w[2][k];
    }
}

// 3-D, pitch a multiple of 4: the sweep (RESID false: out = c + w (b - S c) in
// T) or the residual (RESID true: out = b - S c in the accumulator format),
// with each thread marching zc planes of its four-point row segment.  Per
// plane it keeps the centre row C and the sum A of rows y - 1 and y + 1 (six
// values each, x0 - 1 .. x0 + 4), so each new plane costs three row loads:
//   edges   = A_z[x-1] + A_z[x+1] + C_{z-1}[x-1] + C_{z-1}[x+1]
//             + C_{z+1}[x-1] + C_{z+1}[x+1] + A_{z-1}[x] + A_{z+1}[x],
//   corners = A_{z-1}[x-1] + A_{z-1}[x+1] + A_{z+1}[x-1] + A_{z+1}[x+1],
//   12 S c  = 32 C_z[x] - 2 edges - corners.
// Grid (P/4 / threads, n, ceil(n / zc)).
template <class T, bool RESID>
__global__ __launch_bounds__(kThreads) void k_q1_march4(const T *__restrict__ b, const T *__restrict__ c,
                                                        void *__restrict__ out, int n, int P, int zc, acc_t<T> w) {
    typedef acc_t<T> A;
    const int x0 = 4 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (x0 >= P) return;
    const int y = (int)blockIdx.y + 1;
    const int z0 = (int)blockIdx.z * zc + 1;
    const int z1 = min(z0 + zc - 1, n);
    const bool first = x0 == 0;
    const long Y = P;
    const Grid<3> g{P};
    A Am[6], Cm[6], A0[6], C0[6], Ap[6], Cp[6];
    Q1Plane<T> pl;
    q1_fetch_plane<T>(c + g.at(x0, y, z0 - 1), Y, first, pl);
    q1_widen_plane<T, A>(pl, Am, Cm);
    q1_fetch_plane<T>(c + g.at(x0, y, z0), Y, first, pl);
    q1_widen_plane<T, A>(pl, A0, C0);
    // 4- and 8-byte formats load one plane ahead (c rows of plane z + 1 and b
    // of plane z); the 2-byte ones measured faster loading just in time
    constexpr bool kAhead = sizeof(T) >= 4;
    RawRow<T, 4> bq;
    if constexpr (kAhead) {
        q1_fetch_plane<T>(c + g.at(x0, y, z0 + 1), Y, first, pl);
        fetch_row<T, 4>(b + g.at(x0, y, z0), bq);
    }
    for (int z = z0; z <= z1; ++z) {
        Q1Plane<T> cur;
        RawRow<T, 4> bcur;
        if constexpr (kAhead) {
            cur = pl;
            bcur = bq;
            if (z + 2 <= z1 + 1) q1_fetch_plane<T>(c + g.at(x0, y, z + 2), Y, first, pl);
            if (z + 1 <= z1) fetch_row<T, 4>(b + g.at(x0, y, z + 1), bq);
        } else {
            q1_fetch_plane<T>(c + g.at(x0, y, z + 1), Y, first, cur);
            fetch_row<T, 4>(b + g.at(x0, y, z), bcur);
        }
        q1_widen_plane<T, A>(cur, Ap, Cp);
        const size_t o = g.at(x0, y, z);
        A bv[4];
        widen_row<T, 4>(bcur, bv);
        // the four results are stored with one vector store; x = 0 (first
        // segment) is the ghost and receives zero
        A ra[4];
        T rt[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = i + 1;
            const A e = ((A0[k - 1] + A0[k + 1]) + ((Cm[k - 1] + Cm[k + 1]) + (Cp[k - 1] + Cp[k + 1]))) + (Am[k] + Ap[k]);
            const A cn = (Am[k - 1] + Am[k + 1]) + (Ap[k - 1] + Ap[k + 1]);
            const A sc = fmaT<A>(A(32), C0[k], -fmaT<A>(A(2), e, cn)) * q1_scale<3, A>();
            if (RESID)
                ra[i] = (i == 0 && first) ? A(0) : bv[i] - sc;
            else
                rt[i] = (i == 0 && first) ? zero_of<T>() : Store<T>::from_acc(fmaT<A>(w, bv[i] - sc, C0[k]));
        }
        if (RESID)
            store_row<A, 4>(static_cast<A *>(out) + o, ra);
        else
            store_row<T, 4>(static_cast<T *>(out) + o, rt);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            Am[k] = A0[k], Cm[k] = C0[k];
            A0[k] = Ap[k], C0[k] = Cp[k];
        }
    }
}

// The FP64 update (as k_q1_outer) in the marching form of k_q1_march4: grid
// (P/4 / threads, n, zgroups), zc planes per thread; one partial per block.
// With a ring (DEFER), the update of U is postponed: the correction is
// copied into ring slot *ctr and alpha into adef[*ctr] (U is not touched).
struct Q1Ring {
    void *cd;            // slots of cstride elements in the level format
    size_t cstride;
    double *adef;
    const int *ctr;
};

template <class T, bool DEFER>
__global__ __launch_bounds__(kThreads) void k_q1_outer_march(const T *__restrict__ c, double *__restrict__ R,
                                                             double *__restrict__ U, const double *__restrict__ scal,
                                                             double f, int n, int P, int zc,
                                                             double *__restrict__ part, Q1Ring ring) {
    typedef double A;
    __shared__ double red[8];
    const double a = scal[0];
    T *cd = nullptr;
    if constexpr (DEFER) {
        const int slot = *ring.ctr;
        cd = static_cast<T *>(ring.cd) + (size_t)slot * ring.cstride;
        if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) ring.adef[slot] = a;
    }
    double ss = 0.0, mx = 0.0;
    const int x0 = 4 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int y = (int)blockIdx.y + 1;
    const int z0 = (int)blockIdx.z * zc + 1;
    const int z1 = min(z0 + zc - 1, n);
    if (x0 < P && z0 <= n) {
        const bool first = x0 == 0;
        const long Y = P;
        const Grid<3> g{P};
        A Am[6], Cm[6], A0[6], C0[6], Ap[6], Cp[6];
        Q1Plane<T> pl;
        q1_fetch_plane<T>(c + g.at(x0, y, z0 - 1), Y, first, pl);
        q1_widen_plane<T, A>(pl, Am, Cm);
        q1_fetch_plane<T>(c + g.at(x0, y, z0), Y, first, pl);
        q1_widen_plane<T, A>(pl, A0, C0);
        // 4- and 8-byte formats load one plane ahead (c rows of plane z + 1, R
        // and U of plane z); the 2-byte ones measured faster loading just in time
        constexpr bool kAhead = sizeof(T) >= 4;
        RawRow<double, 4> rq, uq;
        if constexpr (kAhead) {
            q1_fetch_plane<T>(c + g.at(x0, y, z0 + 1), Y, first, pl);
            fetch_row<double, 4>(R + g.at(x0, y, z0), rq);
            if constexpr (!DEFER) fetch_row<double, 4>(U + g.at(x0, y, z0), uq);
        }
        for (int z = z0; z <= z1; ++z) {
            Q1Plane<T> cur;
            RawRow<double, 4> rcur, ucur;
            if constexpr (kAhead) {
                cur = pl;
                rcur = rq;
                if constexpr (!DEFER) ucur = uq;
                if (z + 2 <= z1 + 1) q1_fetch_plane<T>(c + g.at(x0, y, z + 2), Y, first, pl);
                if (z + 1 <= z1) {
                    fetch_row<double, 4>(R + g.at(x0, y, z + 1), rq);
                    if constexpr (!DEFER) fetch_row<double, 4>(U + g.at(x0, y, z + 1), uq);
                }
            } else {
                q1_fetch_plane<T>(c + g.at(x0, y, z + 1), Y, first, cur);
                fetch_row<double, 4>(R + g.at(x0, y, z), rcur);
                if constexpr (!DEFER) fetch_row<double, 4>(U + g.at(x0, y, z), ucur);
            }
            q1_widen_plane<T, A>(cur, Ap, Cp);
            const size_t o = g.at(x0, y, z);
            A rv[4], uv[4] = {};
            widen_row<double, 4>(rcur, rv);
            if constexpr (!DEFER) widen_row<double, 4>(ucur, uv);
            // one vector store each for R and U; x = 0 (first segment) is the
            // ghost: zero, which adds nothing to the norms
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = i + 1;
                const A e =
                    ((A0[k - 1] + A0[k + 1]) + ((Cm[k - 1] + Cm[k + 1]) + (Cp[k - 1] + Cp[k + 1]))) + (Am[k] + Ap[k]);
                const A cn = (Am[k - 1] + Am[k + 1]) + (Ap[k - 1] + Ap[k + 1]);
                const A sc = fmaT<A>(A(32), C0[k], -fmaT<A>(A(2), e, cn)) * q1_scale<3, A>();
                const bool ghost = i == 0 && first;
                const double r = ghost ? 0.0 : fmaT<double>(-a, sc, rv[i]);
                uv[i] = ghost ? 0.0 : fmaT<double>(a * f, C0[k], uv[i]);
                rv[i] = r;
                ss += r * r;
                mx = nanmax(mx, fabs(r));
            }
            store_row<double, 4>(R + o, rv);
            if constexpr (DEFER) {
                T cv[4];  // the correction itself (values of T: exact)
#pragma unroll
                for (int i = 0; i < 4; ++i) cv[i] = (i == 0 && first) ? zero_of<T>() : store_as<T>(C0[i + 1]);
                store_row<T, 4>(cd + o, cv);
            } else {
                store_row<double, 4>(U + o, uv);
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                Am[k] = A0[k], Cm[k] = C0[k];
                A0[k] = Ap[k], C0[k] = Cp[k];
            }
        }
    }
    block_reduce(ss, mx, red);
    if (threadIdx.x == 0) {
        const unsigned b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[2 * b] = ss;
        part[2 * b + 1] = mx;
    }
}

// The marching Q1 kernels with each plane's rows staged in LDS (3-D, pitch a
// multiple of 4).  A block owns TY consecutive rows (threads of row g: x0 = 4 t
// for t < P/4) of zc planes; the rows above and below (g = 0, TY + 1) are
// loaded by their own threads and only written to LDS.  Every plane is read
// from memory once per block row and stored whole in LDS (x = 0 and the ghost
// after a row's last point included), one plane ahead: the thread then forms
// the centre row C and the row sum A = row (y - 1) + row (y + 1) of that plane
// for x0 - 1 .. x0 + 4 from LDS, with the same sums as k_q1_march4, so the
// results are identical.  MODE 0: the sweep (out = c + w (b - S c) in T),
// 1: the residual (out = b - S c in the accumulator format), 2: the FP64
// update (R -= alpha S c; U += alpha f c, or the correction into the ring),
// 3: the FP64 residual r = b - f S c of the iterate c = u from the dense b
// (n x n x n, x fastest) into R, u copied to the dense out (if not null).
// Modes 2 and 3 write one (sum r^2, max |r|) partial per block, and mode 3
// zeros for blocks gridDim.x .. nparts - 1 (the count the caller reduces).
// Mode 4: the residual of mode 1 restricted at once (full weighting into the
// coarse b, format TC, at out): TY (even) owned rows y0 .. y0+TY-1 and the
// row after them, whose residuals the coarse rows (y0+1)/2 .. (y0+TY-1)/2
// need, zc (even) owned planes and the plane after them; each plane's
// residual rows go to LDS (two slots), and after the plane's barrier the
// coarse threads form the x and y sums and carry the z sums in registers, in
// the order of k_q1_restrict (the same result).
template <class T, int MODE, bool DEFER = false, class TC = T>
__global__ __launch_bounds__(1024) void k_q1_lds(const T *__restrict__ b, const T *__restrict__ c,
                                                 void *__restrict__ out, int n, int P, int TY, int zc, int ytiles,
                                                 acc_t<T> w, double *__restrict__ R, double *__restrict__ U,
                                                 const double *__restrict__ scal, double f, double *__restrict__ part,
                                                 Q1Ring ring, int nparts) {
    static_assert(MODE != 3 || sizeof(T) == 8, "the final residual is formed from the FP64 u");
    typedef typename std::conditional<MODE == 2 || MODE == 3, double, acc_t<T>>::type A;
    constexpr bool FR = MODE == 4;  // residual + restriction
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[32];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int TX = P / 4, G = TY + (FR ? 3 : 2);
    const size_t slot = (size_t)G * P + 8;  // G rows and the ghost after the last one
    // mode 4: the residual rows of a plane, two slots after the c slots
    A *rbuf = reinterpret_cast<A *>(smem_raw + ((2 * slot * sizeof(T) + 15) & ~(size_t)15));
    const size_t rslot = (size_t)(TY + 1) * P;
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int yt = blk % ytiles, zch = blk / ytiles;
    const int y0 = 1 + yt * TY;
    const int z0 = 1 + zch * zc, z1 = min(z0 + zc - (FR ? 0 : 1), n);
    const int tx = (int)threadIdx.x % TX, gi = (int)threadIdx.x / TX;
    const int x0 = 4 * tx;
    const int y = y0 - 1 + gi;
    const bool row_in = y >= 1 && y <= n;  // other rows are zero ghosts
    const bool outr = gi >= 1 && gi <= TY + (FR ? 1 : 0) && y <= n;
    A pm = A(0), p0 = A(0);  // mode 4: the coarse thread's y/x sums of planes 2Z - 1 and 2Z
    const bool first = x0 == 0;
    const Grid<3> g{P};
    double ss = 0.0, mx = 0.0;
    T *cd = nullptr;
    double a = 0.0;
    if constexpr (MODE == 2) {
        a = scal[0];
        if constexpr (DEFER) {
            const int s = *ring.ctr;
            cd = static_cast<T *>(ring.cd) + (size_t)s * ring.cstride;
            if (blockIdx.x == 0 && threadIdx.x == 0) ring.adef[s] = a;
        }
    }
    for (int i = threadIdx.x; i < 2 * 8; i += blockDim.x) lds[(i / 8) * slot + (size_t)G * P + (i % 8)] = zero_of<T>();
    auto fetch = [&](int z, RawRow<T, 4> &r) {
        if (row_in) fetch_row<T, 4>(c + g.at(x0, y, z), r);
        else zero_row(r);
    };
    auto publish = [&](int s, const RawRow<T, 4> &r) {
        typedef typename RawRow<T, 4>::C C;
        C *dst = reinterpret_cast<C *>(lds + (size_t)s * slot + (size_t)gi * P + x0);
#pragma unroll
        for (int j = 0; j < RawRow<T, 4>::B / RawRow<T, 4>::CB; ++j) dst[j] = r.c[j];
    };
    // C and A of the plane in slot s for this thread's segment (out rows only)
    auto rows = [&](int s, A (&Av)[6], A (&Cv)[6]) {
        const T *base = lds + (size_t)s * slot + (size_t)gi * P + x0;
        auto row6 = [&](const T *r, A (&v)[6]) {
            A m[4];
            load_row<T, 4>(r, m);
            v[0] = (A)widen(r[first ? 0 : -1]);
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i + 1] = m[i];
            v[5] = (A)widen(r[4]);
        };
        A sv[6], tv[6];
        row6(base, Cv);
        row6(base - P, sv);
        row6(base + P, tv);
#pragma unroll
        for (int k = 0; k < 6; ++k) Av[k] = sv[k] + tv[k];
    };
    A Am[6], Cm[6], A0[6], C0[6], Ap[6], Cp[6];
    RawRow<T, 4> rr;
    fetch(z0 - 1, rr);
    publish(0, rr);
    fetch(z0, rr);
    __syncthreads();
    if (outr) rows(0, Am, Cm);
    publish(1, rr);
    fetch(z0 + 1, rr);
    __syncthreads();
    if (outr) rows(1, A0, C0);
    publish(0, rr);  // slot 0's plane z0 - 1 was read before the last barrier
    if (z0 + 2 <= z1 + 1) fetch(z0 + 2, rr);
    constexpr bool READS_B = MODE <= 1 || MODE == 4;
    RawRow<T, 4> bq;
    if (READS_B && outr) fetch_row<T, 4>(b + g.at(x0, y, z0), bq);
    RawRow<double, 4> rq, uq;
    if (MODE == 2 && outr) {
        fetch_row<double, 4>(R + g.at(x0, y, z0), rq);
        if (!DEFER) fetch_row<double, 4>(U + g.at(x0, y, z0), uq);
    }
    __syncthreads();
    for (int z = z0; z <= z1; ++z) {
        const int it = z - z0;
        const int sp = it & 1;  // slot of plane z + 1
        RawRow<T, 4> bcur = bq;
        RawRow<double, 4> rcur = rq, ucur = uq;
        if (outr) {
            rows(sp, Ap, Cp);
            if (z + 1 <= z1) {
                if (READS_B) fetch_row<T, 4>(b + g.at(x0, y, z + 1), bq);
                if (MODE == 2) {
                    fetch_row<double, 4>(R + g.at(x0, y, z + 1), rq);
                    if (!DEFER) fetch_row<double, 4>(U + g.at(x0, y, z + 1), uq);
                }
            }
            const size_t o = g.at(x0, y, z);
            A sc[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = i + 1;
                const A e =
                    ((A0[k - 1] + A0[k + 1]) + ((Cm[k - 1] + Cm[k + 1]) + (Cp[k - 1] + Cp[k + 1]))) + (Am[k] + Ap[k]);
                const A cn = (Am[k - 1] + Am[k + 1]) + (Ap[k - 1] + Ap[k + 1]);
                sc[i] = fmaT<A>(A(32), C0[k], -fmaT<A>(A(2), e, cn)) * q1_scale<3, A>();
            }
            if constexpr (MODE == 0) {
                A bv[4];
                widen_row<T, 4>(bcur, bv);
                T ov[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    ov[i] = (i == 0 && first) ? zero_of<T>() : Store<T>::from_acc(fmaT<A>(w, bv[i] - sc[i], C0[i + 1]));
                store_row<T, 4>(static_cast<T *>(out) + o, ov);
            } else if constexpr (MODE == 1 || MODE == 4) {
                A bv[4];
                widen_row<T, 4>(bcur, bv);
                A ov[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) ov[i] = (i == 0 && first) ? A(0) : bv[i] - sc[i];
                if constexpr (MODE == 1) store_row<A, 4>(static_cast<A *>(out) + o, ov);
                else store_row<A, 4>(rbuf + (size_t)(it & 1) * rslot + (size_t)(gi - 1) * P + x0, ov);
            } else if constexpr (MODE == 3) {
                // dense b and out: point (x, y, z) at ((z-1) n + (y-1)) n + x-1
                // (the ghost x = 0 reads the row's first point and drops it)
                const size_t d = ((size_t)(z - 1) * n + (y - 1)) * n;
                double rv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool ghost = i == 0 && first;
                    const size_t at = d + (size_t)(ghost ? 0 : x0 + i - 1);
                    const double bv = reinterpret_cast<const double *>(b)[at];
                    const double r = ghost ? 0.0 : bv - f * sc[i];
                    rv[i] = r;
                    ss += r * r;
                    mx = nanmax(mx, fabs(r));
                    if (out && !ghost) static_cast<double *>(out)[at] = C0[i + 1];
                }
                store_row<double, 4>(R + o, rv);
            } else {
                double rv[4], uv[4] = {};
                widen_row<double, 4>(rcur, rv);
                if (!DEFER) widen_row<double, 4>(ucur, uv);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool ghost = i == 0 && first;
                    const double r = ghost ? 0.0 : fmaT<double>(-a, sc[i], rv[i]);
                    uv[i] = ghost ? 0.0 : fmaT<double>(a * f, C0[i + 1], uv[i]);
                    rv[i] = r;
                    ss += r * r;
                    mx = nanmax(mx, fabs(r));
                }
                store_row<double, 4>(R + o, rv);
                if constexpr (DEFER) {
                    T cv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) cv[i] = (i == 0 && first) ? zero_of<T>() : store_as<T>(C0[i + 1]);
                    store_row<T, 4>(cd + o, cv);
                } else {
                    store_row<double, 4>(U + o, uv);
                }
            }
        }
        // plane z + 2 into the slot plane z occupied (read before the last barrier)
        if (z + 1 <= z1) {
            publish(sp ^ 1, rr);
            if (z + 3 <= z1 + 1) fetch(z + 3, rr);
        }
        __syncthreads();
        if constexpr (FR) {
            // coarse point (X, Y) of this tile: fine rows 2Y - 1 .. 2Y + 1 are
            // residual rows 2j .. 2j + 2 of the slot written before the barrier
            const int Pc = (n - 1) / 2 + 1, nc = Pc - 1;
            const int t = (int)threadIdx.x, j = t / Pc, X = t - j * Pc, Y = (y0 + 1) / 2 + j;
            if (j < TY / 2 && X >= 1 && Y <= nc) {
                const A *q = rbuf + (size_t)(it & 1) * rslot + (size_t)(2 * j) * P + 2 * X;
                auto row = [&](const A *v) -> A { return (v[-1] + v[1]) + A(2) * v[0]; };
                const A py = (row(q) + row(q + 2 * P)) + A(2) * row(q + P);
                if (z & 1) {
                    if (z > z0) {
                        A sum = (pm + py) + A(2) * p0;
                        sum *= A(1.0 / 64.0);
                        static_cast<TC *>(out)[Grid<3>{Pc}.at(X, Y, (z - 1) / 2)] = store_as<TC>(sum);
                    }
                    pm = py;
                } else {
                    p0 = py;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            Am[k] = A0[k], Cm[k] = C0[k];
            A0[k] = Ap[k], C0[k] = Cp[k];
        }
    }
    if constexpr (MODE == 2 || MODE == 3) {
        block_reduce(ss, mx, red);
        if (threadIdx.x == 0) {
            part[2 * blockIdx.x] = ss;
            part[2 * blockIdx.x + 1] = mx;
            if constexpr (MODE == 3)
                for (int i = blockIdx.x + gridDim.x; i < nparts; i += gridDim.x) part[2 * i] = part[2 * i + 1] = 0.0;
        }
    }
}

// Full weighting of r at coarse point (X, Y, Z), whose fine twin is
// (2X, 2Y, 2Z): 1-D weights 1, 2, 1 summed exactly and scaled by 4^-D.
template <int D, class A, class TC>
__global__ __launch_bounds__(kThreads) void k_q1_restrict(const A *__restrict__ r, TC *__restrict__ bc, int nc,
                                                          int Pf, int Pc, unsigned Nc) {
    const unsigned i = q1_index(1);
    if (i >= Nc) return;
    int X, Y, Z;
    const size_t oc = q1_at<D>(i, nc, Pc, X, Y, Z);
    const Grid<D> gf{Pf};
    const long o = (long)(D == 3 ? gf.at(2 * X, 2 * Y, 2 * Z) : gf.at(2 * X, 0, 2 * Z));
    const long Yf = Pf, Zf = (long)Pf * Pf;
    auto row = [&](long c0) -> A { return (r[c0 - 1] + r[c0 + 1]) + A(2) * r[c0]; };
    A s;
    if (D == 2) {
        s = (row(o - Yf) + row(o + Yf)) + A(2) * row(o);
        s *= A(1.0 / 16.0);
    } else {
        auto plane = [&](long c0) -> A { return (row(c0 - Yf) + row(c0 + Yf)) + A(2) * row(c0); };
        s = (plane(o - Zf) + plane(o + Zf)) + A(2) * plane(o);
        s *= A(1.0 / 64.0);
    }
    bc[oc] = store_as<TC>(s);
}

// c += 4 P ec (linear interpolation of the coarse correction) in place, in W:
// along each axis an even fine index 2X copies coarse X, an odd one averages
// coarse (x-1)/2 and (x+1)/2 (ghosts hold zero).  A segment's fine points
// x0 .. x0+3 need coarse x from x0/2 to x0/2 + 2 (x0 odd).
template <int D, class TF, class TC>
__global__ __launch_bounds__(kThreads) void k_q1_prolong_add(TF *__restrict__ c, const TC *__restrict__ ec, int n,
                                                             int P, int Pc, unsigned NS) {
    typedef typename std::conditional<sizeof(acc_t<TF>) >= sizeof(acc_t<TC>), acc_t<TF>, acc_t<TC>>::type W;
    constexpr int K = kV / 2 + 1;
    const unsigned t = q1_index(1);
    if (t >= NS) return;
    const unsigned ns = q1_segs_per_row(n);
    const unsigned row = t / ns;
    const int x0 = 1 + kV * (int)(t - row * ns);
    const int y = D == 3 ? (int)(row % (unsigned)n) + 1 : 0;
    const int z = D == 3 ? (int)(row / (unsigned)n) + 1 : (int)row + 1;
    const long o = D == 3 ? (long)Grid<3>{P}.at(x0, y, z) : (long)Grid<2>{P}.at(x0, 0, z);
    const Grid<D> gc{Pc};
    const int cx = x0 >> 1;
    // s2[k]: coarse value at x = cx + k summed over the (up to) 2 x 2 coarse
    // rows around the fine row, each axis counting an aligned row twice
    W s2[K];
    const int z0 = z >> 1, z1 = (z + 1) >> 1;
    if (D == 2) {
        const long b0 = (long)gc.at(cx, 0, z0), b1 = (long)gc.at(cx, 0, z1);
#pragma unroll
        for (int k = 0; k < K; ++k) s2[k] = (W)widen(ec[b0 + k]) + (W)widen(ec[b1 + k]);
    } else {
        const int y0 = y >> 1, y1 = (y + 1) >> 1;
        const long b00 = (long)gc.at(cx, y0, z0), b10 = (long)gc.at(cx, y1, z0);
        const long b01 = (long)gc.at(cx, y0, z1), b11 = (long)gc.at(cx, y1, z1);
#pragma unroll
        for (int k = 0; k < K; ++k)
            s2[k] = ((W)widen(ec[b00 + k]) + (W)widen(ec[b10 + k])) + ((W)widen(ec[b01 + k]) + (W)widen(ec[b11 + k]));
    }
#pragma unroll
    for (int i = 0; i < kV; ++i) {
        const int x = x0 + i;
        if (x > n) break;
        // 2^D times the interpolant; 4 P ec = that * 4 / 2^D
        W s = s2[(x >> 1) - cx] + s2[((x + 1) >> 1) - cx];
        s *= W(D == 3 ? 0.5 : 1.0);
        c[o + i] = store_as<TF>((W)widen(c[o + i]) + s);
    }
}

// The same on a level whose pitch P is a multiple of 4: segment t covers x0
// = 4j .. 4j + 3 of one row (x = 0, the ghost, keeps its value), so c is read
// and written with one vector access; coarse x from 2j to 2j + 2.  Same sums
// per point as k_q1_prolong_add.
template <int D, class TF, class TC>
__global__ __launch_bounds__(kThreads) void k_q1_prolong_add4(TF *__restrict__ c, const TC *__restrict__ ec, int n,
                                                              int P, int Pc, unsigned NS) {
    typedef typename std::conditional<sizeof(acc_t<TF>) >= sizeof(acc_t<TC>), acc_t<TF>, acc_t<TC>>::type W;
    const unsigned t = q1_index(1);
    if (t >= NS) return;
    const unsigned ns = (unsigned)P / 4;
    const unsigned row = t / ns;
    const int x0 = 4 * (int)(t - row * ns);
    const int y = D == 3 ? (int)(row % (unsigned)n) + 1 : 0;
    const int z = D == 3 ? (int)(row / (unsigned)n) + 1 : (int)row + 1;
    const size_t o = D == 3 ? Grid<3>{P}.at(x0, y, z) : Grid<2>{P}.at(x0, 0, z);
    const Grid<D> gc{Pc};
    const int cx = x0 >> 1;
    auto coarse3 = [&](size_t b, W (&v)[3]) {
        TC two[2];
        load_raw<TC, 2>(ec + b, two);  // cx is even: an aligned pair
        v[0] = (W)widen(two[0]);
        v[1] = (W)widen(two[1]);
        v[2] = (W)widen(ec[b + 2]);
    };
    W s2[3];
    const int z0 = z >> 1, z1 = (z + 1) >> 1;
    if (D == 2) {
        W a[3], bb[3];
        coarse3(gc.at(cx, 0, z0), a);
        coarse3(gc.at(cx, 0, z1), bb);
#pragma unroll
        for (int k = 0; k < 3; ++k) s2[k] = a[k] + bb[k];
    } else {
        const int y0 = y >> 1, y1 = (y + 1) >> 1;
        W v00[3], v10[3], v01[3], v11[3];
        coarse3(gc.at(cx, y0, z0), v00);
        coarse3(gc.at(cx, y1, z0), v10);
        coarse3(gc.at(cx, y0, z1), v01);
        coarse3(gc.at(cx, y1, z1), v11);
#pragma unroll
        for (int k = 0; k < 3; ++k) s2[k] = (v00[k] + v10[k]) + (v01[k] + v11[k]);
    }
    TF cv[4];
    load_raw<TF, 4>(c + o, cv);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int x = x0 + i;
        if (x == 0) continue;  // the ghost
        W sx = s2[(x >> 1) - cx] + s2[((x + 1) >> 1) - cx];
        sx *= W(D == 3 ? 0.5 : 1.0);
        cv[i] = store_as<TF>((W)widen(cv[i]) + sx);
    }
    store_row<TF, 4>(c + o, cv);
}

// Finest-level update of a refinement step in FP64: U += alpha f c and
// R -= alpha S c (the recursively updated residual of Algorithm 2), f =
// h^(2-D) undoing the grid scaling; partial sum of squares and max |R| per block.
template <int D, class T, bool DEFER>
__global__ __launch_bounds__(kThreads) void k_q1_outer(const T *__restrict__ c, double *__restrict__ R,
                                                       double *__restrict__ U, const double *__restrict__ scal,
                                                       double f, int n, int P, double *__restrict__ part, Q1Ring ring) {
    // grid (x blocks, gy): a thread keeps its x and walks the rows
    // blockIdx.y, blockIdx.y + gy, ... (row = y + n z in 3-D)
    __shared__ double red[8];
    const double a = scal[0];
    T *cd = nullptr;
    if constexpr (DEFER) {
        const int slot = *ring.ctr;
        cd = static_cast<T *>(ring.cd) + (size_t)slot * ring.cstride;
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) ring.adef[slot] = a;
    }
    double ss = 0.0, mx = 0.0;
    const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x) + 1;
    const unsigned rows = D == 3 ? (unsigned)n * n : (unsigned)n;
    if (x <= n) {
        for (unsigned row = blockIdx.y; row < rows; row += gridDim.y) {
            const size_t o = D == 3 ? Grid<3>{P}.at(x, (int)(row % (unsigned)n) + 1, (int)(row / (unsigned)n) + 1)
                                    : Grid<2>{P}.at(x, 0, (int)row + 1);
            const double sc = q1_weighted<D, double>(c, o, P) * q1_scale<D, double>();
            const double r = fmaT<double>(-a, sc, R[o]);
            R[o] = r;
            if constexpr (DEFER)
                cd[o] = c[o];
            else
                U[o] = fmaT<double>(a * f, (double)widen(c[o]), U[o]);
            ss += r * r;
            mx = nanmax(mx, fabs(r));
        }
    }
    block_reduce(ss, mx, red);
    if (threadIdx.x == 0) {
        const unsigned b = blockIdx.y * gridDim.x + blockIdx.x;
        part[2 * b] = ss;
        part[2 * b + 1] = mx;
    }
}

// r = b - hd S U (hd = h^(D-2)) from the dense right-hand side b; without U,
// r = b.  Optionally writes r into the padded R and U into the dense uout;
// partial sum of squares and max |r| per block.
template <int D>
__global__ __launch_bounds__(kThreads) void k_q1_resid_flat(const double *__restrict__ b, const double *__restrict__ U,
                                                            double *__restrict__ R, double *__restrict__ uout, int n,
                                                            int P, unsigned N, double hd, double *__restrict__ part) {
    __shared__ double red[8];
    double ss = 0.0, mx = 0.0;
    for (unsigned i = blockIdx.x * kThreads + threadIdx.x; i < N; i += gridDim.x * kThreads) {
        int x, y, z;
        const size_t o = q1_at<D>(i, n, P, x, y, z);
        double r = b[i];
        if (U) {
            r -= hd * (q1_weighted<D, double>(U, o, P) * q1_scale<D, double>());
            if (uout) uout[i] = U[o];
        }
        if (R) R[o] = r;
        ss += r * r;
        mx = nanmax(mx, fabs(r));
    }
    block_reduce(ss, mx, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss;
        part[2 * blockIdx.x + 1] = mx;
    }
}

// One-point base level: S c = b with S = 8/3.
template <int D, class T> __global__ void k_q1_coarse(const T *__restrict__ b, T *__restrict__ c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        typedef acc_t<T> A;
        const int i = D == 3 ? 7 : 3;
        c[i] = Store<T>::from_acc((A)widen(b[i]) * A(0.375));
    }
}

unsigned npoints(int D, int n) { return D == 3 ? (unsigned)n * n * n : (unsigned)n * n; }
// Threads along x of the point-mapped kernels, and their grid.
int q1_bx(int n) { return n > 128 ? 256 : n > 64 ? 128 : 64; }
// Four-point forms: P/4 threads per row.
int q1_bx4(int P) { return P / 4 > 128 ? 256 : P / 4 > 64 ? 128 : 64; }
dim3 q1_grid4(int D, int n, int P) {
    const unsigned bx = (unsigned)((P / 4 + q1_bx4(P) - 1) / q1_bx4(P));
    return D == 3 ? dim3(bx, (unsigned)n, (unsigned)n) : dim3(bx, (unsigned)n, 1);
}
// Planes marched by one thread of k_q1_march4, and its grid.
constexpr int kMarchZ = 16;
dim3 q1_grid4z(int n, int P) {
    const unsigned bx = (unsigned)((P / 4 + q1_bx4(P) - 1) / q1_bx4(P));
    return dim3(bx, (unsigned)n, (unsigned)((n + kMarchZ - 1) / kMarchZ));
}
dim3 q1_grid(int D, int n) {
    const unsigned bx = (unsigned)((n + q1_bx(n) - 1) / q1_bx(n));
    return D == 3 ? dim3(bx, (unsigned)n, (unsigned)n) : dim3(bx, (unsigned)n, 1);
}
int nblocks(unsigned N) { return (int)((N + kThreads - 1) / kThreads); }

template <class T>
hipError_t first_t(int D, int n, int P, const void *b, const double *R, const double *scal, void *bout, void *cout,
                   double omega, hipStream_t st) {
    typedef acc_t<T> A;
    const A w = (A)(omega * 0.375);
    const T *bb = static_cast<const T *>(b);
    T *bo = static_cast<T *>(bout), *co = static_cast<T *>(cout);
    if (P % 4 == 0) {
        const long segs = (long)(P / 4) * (D == 3 ? (long)n * n : (long)n);
        const unsigned blocks = (unsigned)((segs + kThreads - 1) / kThreads);
#define MG_Q1F4(DD, FR)                                                                                        \
    hipLaunchKernelGGL((k_q1_first4<DD, T, FR>), dim3(blocks), dim3(kThreads), 0, st, bb, R, scal, bo, co, n, P, w)
        if (D == 3) {
            if (R) MG_Q1F4(3, true);
            else MG_Q1F4(3, false);
        } else {
            if (R) MG_Q1F4(2, true);
            else MG_Q1F4(2, false);
        }
#undef MG_Q1F4
        return hipGetLastError();
    }
    if (R) {
        if (D == 3)
            hipLaunchKernelGGL((k_q1_first<3, T, true>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, bb, R, scal, bo, co,
                               n, P, w);
        else
            hipLaunchKernelGGL((k_q1_first<2, T, true>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, bb, R, scal, bo, co,
                               n, P, w);
    } else {
        if (D == 3)
            hipLaunchKernelGGL((k_q1_first<3, T, false>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, bb, R, scal, bo,
                               co, n, P, w);
        else
            hipLaunchKernelGGL((k_q1_first<2, T, false>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, bb, R, scal, bo,
                               co, n, P, w);
    }
    return hipGetLastError();
}

// Shape of k_q1_lds on a 3-D level of pitch P (a multiple of 4), o.ty rows
// and o.zc planes, or with o.ty = 0 the built-in choice: the most rows per
// block that 1024 threads and 64 KB of LDS allow, up to 6, and up to 16
// planes, fewer where that leaves under about four blocks per CU.
struct Q1LdsShape {
    int TY, zc, ytiles, blocks;
    size_t lds;
};
Q1LdsShape q1_lds_shape(int n, int P, size_t sb, const Q1Shape &o = Q1Shape{}) {
    Q1LdsShape s{};
    const int TX = P / 4;
    if (o.ty > 0) {
        s.TY = o.ty;
        s.zc = o.zc;
    } else {
        s.TY = std::min(6, 1024 / TX - 2);
        while (s.TY > 1 && 2 * (((size_t)s.TY + 2) * P + 8) * sb > 65536 - 512) --s.TY;
        s.zc = std::max(2, std::min(16, (int)(((long)n * ((n + s.TY - 1) / s.TY) + 1023) / 1024)));
        s.zc = std::min(s.zc, n);
    }
    s.ytiles = (n + s.TY - 1) / s.TY;
    s.blocks = s.zc >= 1 ? s.ytiles * ((n + s.zc - 1) / s.zc) : 0;
    s.lds = 2 * (((size_t)s.TY + 2) * P + 8) * sb;
    return s;
}
// Whether the 3-D level takes k_q1_lds (2-byte format, pitch a multiple of 4,
// room for two rows of threads plus one owned row, and no more blocks than the
// update's partials allow) in shape o.
bool q1_lds_ok(int n, int P, size_t sb, const Q1Shape &o = Q1Shape{}) {
    // the 2-byte formats (the 4- and 8-byte ones measured faster marching with
    // their own row loads one plane ahead)
    if (sb != 2 || P % 4 != 0 || P / 4 > 1024 / 3) return false;
    const Q1LdsShape s = q1_lds_shape(n, P, sb, o);
    return s.TY >= 1 && (s.TY + 2) * (P / 4) <= 1024 && s.lds <= 65536 - 512 && s.zc >= 1 && s.zc <= n &&
           s.blocks <= flat_blocks((long)npoints(3, n));
}

template <class T, int MODE, bool DEFER = false>
hipError_t q1_lds_launch(int n, int P, const void *b, const void *c, void *out, acc_t<T> w, double *R, double *U,
                         const double *scal, double f, double *part, const Q1Ring &ring, const Q1Shape &o,
                         hipStream_t st) {
    if (!q1_lds_ok(n, P, sizeof(T), o)) return hipErrorInvalidValue;
    const Q1LdsShape s = q1_lds_shape(n, P, sizeof(T), o);
    hipLaunchKernelGGL((k_q1_lds<T, MODE, DEFER>), dim3(s.blocks), dim3((s.TY + 2) * (P / 4)), s.lds, st,
                       static_cast<const T *>(b), static_cast<const T *>(c), out, n, P, s.TY, s.zc, s.ytiles, w, R, U,
                       scal, f, part, ring, s.blocks);
    return hipGetLastError();
}

// Shape of the fused residual + restriction (k_q1_lds mode 4): o.ty fine rows
// and o.zc fine planes per block (both even), or with o.ty = 0 the most rows,
// up to 6, that 1024 threads ((ty + 3) P / 4) and 64 KB of LDS (two slots of
// c rows, two of residual rows in the accumulator format) allow, and planes
// so that the blocks about fill four rounds over the CUs.
Q1LdsShape q1_fr_shape(int n, int P, size_t sb, size_t sa, const Q1Shape &o) {
    Q1LdsShape s{};
    const int TX = P / 4, nc = (n - 1) / 2;
    auto lds = [&](int ty) {
        return ((2 * (((size_t)ty + 3) * P + 8) * sb + 15) & ~(size_t)15) + 2 * ((size_t)ty + 1) * P * sa;
    };
    if (o.ty > 0) {
        s.TY = o.ty;
        s.zc = o.zc;
    } else {
        s.TY = std::min(6, 1024 / TX - 3) & ~1;
        while (s.TY > 2 && lds(s.TY) > 65536 - 512) s.TY -= 2;
        const int yt = s.TY >= 2 ? (nc + s.TY / 2 - 1) / (s.TY / 2) : 1;
        s.zc = 2 * std::max(1, std::min(8, (int)(((long)nc * yt + 1023) / 1024)));
    }
    s.ytiles = s.TY >= 2 ? (nc + s.TY / 2 - 1) / (s.TY / 2) : 0;
    s.blocks = s.zc >= 2 ? s.ytiles * ((nc + s.zc / 2 - 1) / (s.zc / 2)) : 0;
    s.lds = lds(std::max(s.TY, 0));
    return s;
}
bool q1_fr_ok(int n, int P, size_t sb, size_t sa, const Q1Shape &o) {
    if (sb != 2 || P % 4 != 0 || n < 3 || n % 2 == 0 || o.split) return false;
    const Q1LdsShape s = q1_fr_shape(n, P, sb, sa, o);
    return s.TY >= 2 && s.TY % 2 == 0 && (s.TY + 3) * (P / 4) <= 1024 && s.zc >= 2 && s.zc % 2 == 0 &&
           s.zc <= n + 1 && s.lds <= 65536 - 512 && s.blocks >= 1;
}

// The final residual r = b - hd S u of a 3-D level from the dense b (k_q1_lds
// mode 3): FP64 rows in LDS, the built-in shape for 8-byte elements; false
// where it does not apply (pitch, threads, LDS, more blocks than partials).
bool q1_final_lds_ok(int n, int P) {
    if (P % 4 != 0 || P / 4 > 1024 / 3) return false;
    const Q1LdsShape s = q1_lds_shape(n, P, sizeof(double));
    return s.TY >= 1 && (s.TY + 2) * (P / 4) <= 1024 && s.lds <= 65536 - 512 &&
           s.blocks <= flat_blocks((long)npoints(3, n));
}

template <class T>
hipError_t sweep_t(int D, int n, int P, const void *b, const void *c, void *cout, double omega, const Q1Shape &qs,
                   hipStream_t st) {
    typedef acc_t<T> A;
    const A w = (A)(omega * 0.375);
    if (D == 3 && q1_lds_ok(n, P, sizeof(T)))
        return q1_lds_launch<T, 0>(n, P, b, c, cout, w, nullptr, nullptr, nullptr, 0.0, nullptr, Q1Ring{}, qs, st);
    if (P % 4 == 0) {
        const dim3 g4 = q1_grid4(D, n, P);
        if (D == 3)
            hipLaunchKernelGGL((k_q1_march4<T, false>), q1_grid4z(n, P), dim3(q1_bx4(P)), 0, st,
                               static_cast<const T *>(b), static_cast<const T *>(c), cout, n, P, kMarchZ, w);
        else
            hipLaunchKernelGGL((k_q1_sweep4<2, T>), g4, dim3(q1_bx4(P)), 0, st, static_cast<const T *>(b),
                               static_cast<const T *>(c), static_cast<T *>(cout), P, w);
        return hipGetLastError();
    }
    if (D == 3)
        hipLaunchKernelGGL((k_q1_sweep<3, T>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, static_cast<const T *>(b),
                           static_cast<const T *>(c), static_cast<T *>(cout), n, P, w);
    else
        hipLaunchKernelGGL((k_q1_sweep<2, T>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, static_cast<const T *>(b),
                           static_cast<const T *>(c), static_cast<T *>(cout), n, P, w);
    return hipGetLastError();
}

template <class T, class TC>
hipError_t restrict_t(int D, int n, int P, const void *b, const void *c, void *rs, void *bc, const Q1Shape &qs,
                      hipStream_t st) {
    typedef acc_t<T> A;
    const int nc = (n - 1) / 2, Pc = nc + 1;
    const unsigned Nc = npoints(D, nc);
    A *r = static_cast<A *>(rs);
    const bool builtin = qs.ty == 0 && qs.zc == 0;
    if constexpr (sizeof(T) == 2) {  // the levels that take the LDS-staged kernels
        if (D == 3 && q1_lds_ok(n, P, sizeof(T)) && !qs.split &&
            (!builtin || q1_fr_ok(n, P, sizeof(T), sizeof(A), qs))) {
            // residual and restriction in one pass (the fine residual stays in
            // LDS; the built-in shape falls back to two kernels where no tile fits)
            if (!q1_fr_ok(n, P, sizeof(T), sizeof(A), qs)) return hipErrorInvalidValue;
            const Q1LdsShape s = q1_fr_shape(n, P, sizeof(T), sizeof(A), qs);
            hipLaunchKernelGGL((k_q1_lds<T, 4, false, TC>), dim3(s.blocks), dim3((s.TY + 3) * (P / 4)), s.lds, st,
                               static_cast<const T *>(b), static_cast<const T *>(c), bc, n, P, s.TY, s.zc, s.ytiles,
                               A(0), nullptr, nullptr, nullptr, 0.0, nullptr, Q1Ring{}, 0);
            return hipGetLastError();
        }
    }
    if (P % 4 == 0) {
        const dim3 g4 = q1_grid4(D, n, P);
        if (D == 3 && q1_lds_ok(n, P, sizeof(T))) {
            const hipError_t e = q1_lds_launch<T, 1>(n, P, b, c, static_cast<void *>(r), A(0), nullptr, nullptr,
                                                     nullptr, 0.0, nullptr, Q1Ring{}, qs, st);
            if (e != hipSuccess) return e;
        } else if (D == 3)
            hipLaunchKernelGGL((k_q1_march4<T, true>), q1_grid4z(n, P), dim3(q1_bx4(P)), 0, st,
                               static_cast<const T *>(b), static_cast<const T *>(c), static_cast<void *>(r), n, P,
                               kMarchZ, A(0));
        else
            hipLaunchKernelGGL((k_q1_resid4<2, T>), g4, dim3(q1_bx4(P)), 0, st, static_cast<const T *>(b),
                               static_cast<const T *>(c), r, P);
        if (D == 3)
            hipLaunchKernelGGL((k_q1_restrict<3, A, TC>), dim3(nblocks(Nc)), dim3(kThreads), 0, st, r,
                               static_cast<TC *>(bc), nc, P, Pc, Nc);
        else
            hipLaunchKernelGGL((k_q1_restrict<2, A, TC>), dim3(nblocks(Nc)), dim3(kThreads), 0, st, r,
                               static_cast<TC *>(bc), nc, P, Pc, Nc);
        return hipGetLastError();
    }
    if (D == 3) {
        hipLaunchKernelGGL((k_q1_resid<3, T>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, static_cast<const T *>(b),
                           static_cast<const T *>(c), r, n, P);
        hipLaunchKernelGGL((k_q1_restrict<3, A, TC>), dim3(nblocks(Nc)), dim3(kThreads), 0, st, r,
                           static_cast<TC *>(bc), nc, P, Pc, Nc);
    } else {
        hipLaunchKernelGGL((k_q1_resid<2, T>), q1_grid(D, n), dim3(q1_bx(n)), 0, st, static_cast<const T *>(b),
                           static_cast<const T *>(c), r, n, P);
        hipLaunchKernelGGL((k_q1_restrict<2, A, TC>), dim3(nblocks(Nc)), dim3(kThreads), 0, st, r,
                           static_cast<TC *>(bc), nc, P, Pc, Nc);
    }
    return hipGetLastError();
}

template <class TF, class TC>
hipError_t prolong_t(int D, int n, int P, void *c, const void *ec, hipStream_t st) {
    const int Pc = (n - 1) / 2 + 1;
    if (P % 4 == 0) {
        const unsigned N = (unsigned)(P / 4) * (D == 3 ? (unsigned)n * n : (unsigned)n);
        if (D == 3)
            hipLaunchKernelGGL((k_q1_prolong_add4<3, TF, TC>), dim3(nblocks(N)), dim3(kThreads), 0, st,
                               static_cast<TF *>(c), static_cast<const TC *>(ec), n, P, Pc, N);
        else
            hipLaunchKernelGGL((k_q1_prolong_add4<2, TF, TC>), dim3(nblocks(N)), dim3(kThreads), 0, st,
                               static_cast<TF *>(c), static_cast<const TC *>(ec), n, P, Pc, N);
        return hipGetLastError();
    }
    const unsigned N = q1_segs(D, n);
    if (D == 3)
        hipLaunchKernelGGL((k_q1_prolong_add<3, TF, TC>), dim3(nblocks(N)), dim3(kThreads), 0, st,
                           static_cast<TF *>(c), static_cast<const TC *>(ec), n, P, Pc, N);
    else
        hipLaunchKernelGGL((k_q1_prolong_add<2, TF, TC>), dim3(nblocks(N)), dim3(kThreads), 0, st,
                           static_cast<TF *>(c), static_cast<const TC *>(ec), n, P, Pc, N);
    return hipGetLastError();
}

// Grid of the update: q1_bx(n) threads along x, gy row groups, at most
// flat_blocks(points) blocks (= reduction partials) in all.
// The marching update (k_q1_outer_march) serves 3-D levels of pitch a
// multiple of 4 whose (x blocks, n rows) fit the partial budget
// flat_blocks(points); the rest take k_q1_outer.
bool q1_outer_marches(int D, int n) {
    const int P = n + 1;
    if (D != 3 || P % 4 != 0) return false;
    const int xb = (P / 4 + q1_bx4(P) - 1) / q1_bx4(P);
    return xb * n <= flat_blocks((long)npoints(D, n));
}

dim3 q1_outer_grid(int D, int n) {
    const int P = n + 1, cap = flat_blocks((long)npoints(D, n));
    if (q1_outer_marches(D, n)) {
        const int xb = (P / 4 + q1_bx4(P) - 1) / q1_bx4(P);
        return dim3((unsigned)xb, (unsigned)n, (unsigned)std::min(n, cap / (xb * n)));
    }
    const int xb = (n + q1_bx(n) - 1) / q1_bx(n);
    return dim3((unsigned)xb, (unsigned)std::max(1, cap / xb), 1);
}

template <class T, bool DEFER>
hipError_t outer_t(int D, int n, int P, const void *c, double *R, double *U, const double *scal, double f,
                   double *part, const Q1Ring &ring, const Q1Shape &qs, hipStream_t st) {
    if (D == 3 && q1_lds_ok(n, P, sizeof(T)))
        return q1_lds_launch<T, 2, DEFER>(n, P, nullptr, c, nullptr, acc_t<T>(0), R, U, scal, f, part, ring, qs, st);
    const dim3 g = q1_outer_grid(D, n);
    if (q1_outer_marches(D, n)) {
        const int zc = (n + (int)g.z - 1) / (int)g.z;
        hipLaunchKernelGGL((k_q1_outer_march<T, DEFER>), g, dim3(q1_bx4(P)), 0, st, static_cast<const T *>(c), R, U,
                           scal, f, n, P, zc, part, ring);
        return hipGetLastError();
    }
    if (D == 3)
        hipLaunchKernelGGL((k_q1_outer<3, T, DEFER>), g, dim3(q1_bx(n)), 0, st, static_cast<const T *>(c), R, U, scal,
                           f, n, P, part, ring);
    else
        hipLaunchKernelGGL((k_q1_outer<2, T, DEFER>), g, dim3(q1_bx(n)), 0, st, static_cast<const T *>(c), R, U, scal,
                           f, n, P, part, ring);
    return hipGetLastError();
}

}  // namespace

#define Q1_DISPATCH(prec, TT, ...)                 \
    switch (prec) {                                \
    case P_F64: {                                  \
        typedef double TT;                         \
        __VA_ARGS__;                               \
    }                                              \
    case P_F32: {                                  \
        typedef float TT;                          \
        __VA_ARGS__;                               \
    }                                              \
    case P_F16: {                                  \
        typedef f16 TT;                            \
        __VA_ARGS__;                               \
    }                                              \
    case P_BF16: {                                 \
        typedef bf16 TT;                           \
        __VA_ARGS__;                               \
    }                                              \
    default: return hipErrorInvalidValue;          \
    }

size_t q1_resid_bytes(int D, int prec, int P) {
    return level_elems(D, P) * (prec == P_F64 ? sizeof(double) : sizeof(float));
}

bool q1_lds_level(int D, int prec, int n, int P) { return D == 3 && q1_lds_ok(n, P, prec_bytes(prec)); }

namespace {
size_t q1_acc_bytes(int prec) { return prec == P_F64 ? 8 : 4; }
bool q1_fused_restrict(int kernel, const Q1Shape &s) { return kernel == 1 && !s.split; }
}  // namespace

bool q1_shape_ok(int D, int prec, int n, int P, int kernel, const Q1Shape &s) {
    if (s.split != 0 && (s.split != 1 || kernel != 1)) return false;
    if (!q1_lds_level(D, prec, n, P)) return s.ty == 0 && s.zc == 0 && s.split == 0;
    if (s.ty == 0 && s.zc == 0) return true;
    if (s.ty <= 0) return false;
    if (q1_fused_restrict(kernel, s)) return q1_fr_ok(n, P, prec_bytes(prec), q1_acc_bytes(prec), s);
    return q1_lds_ok(n, P, prec_bytes(prec), s);
}

Q1Shape q1_shape_used(int D, int prec, int n, int P, int kernel, const Q1Shape &s) {
    if (!q1_lds_level(D, prec, n, P)) return Q1Shape{};
    const bool builtin = s.ty == 0 && s.zc == 0;
    if (q1_fused_restrict(kernel, s) &&
        (!builtin || q1_fr_ok(n, P, prec_bytes(prec), q1_acc_bytes(prec), s))) {
        const Q1LdsShape u = q1_fr_shape(n, P, prec_bytes(prec), q1_acc_bytes(prec), s);
        return Q1Shape{u.TY, u.zc, 0};
    }
    const Q1LdsShape u = q1_lds_shape(n, P, prec_bytes(prec), s);
    return Q1Shape{u.TY, u.zc, kernel == 1 ? 1 : 0};
}

int q1_outer_blocks(int D, int n, int prec, const Q1Shape &qs) {
    const int P = n + 1;
    if (D == 3 && q1_lds_ok(n, P, prec_bytes(prec))) return q1_lds_shape(n, P, prec_bytes(prec), qs).blocks;
    const dim3 g = q1_outer_grid(D, n);
    return (int)(g.x * g.y * g.z);
}

hipError_t launch_q1_first(int D, int prec, int n, int P, const void *b, const double *R, const double *scal,
                           void *b_out, void *c_out, double omega, hipStream_t st) {
    Q1_DISPATCH(prec, TT, return first_t<TT>(D, n, P, b, R, scal, b_out, c_out, omega, st));
}

hipError_t launch_q1_sweep(int D, int prec, int n, int P, const void *b, const void *c, void *c_out, double omega,
                           hipStream_t st, const Q1Shape &s) {
    Q1_DISPATCH(prec, TT, return sweep_t<TT>(D, n, P, b, c, c_out, omega, s, st));
}

hipError_t launch_q1_restrict(int D, int pf, int pc, int n, int P, const void *b, const void *c, void *rs, void *bc,
                              hipStream_t st, const Q1Shape &s) {
    if (n < 3 || n % 2 == 0) return hipErrorInvalidValue;
    Q1_DISPATCH(pf, TF, Q1_DISPATCH(pc, TC, return (restrict_t<TF, TC>(D, n, P, b, c, rs, bc, s, st))));
}

hipError_t launch_q1_prolong(int D, int pf, int pc, int n, int P, const void *c, const void *ec, const void *b,
                             void *c_out, double omega, hipStream_t st, const Q1Shape &s) {
    if (n < 3 || n % 2 == 0) return hipErrorInvalidValue;
    hipError_t e = hipErrorInvalidValue;
    Q1_DISPATCH(pf, TF, Q1_DISPATCH(pc, TC, e = (prolong_t<TF, TC>(D, n, P, const_cast<void *>(c), ec, st)); break);
                break);
    if (e != hipSuccess) return e;
    return launch_q1_sweep(D, pf, n, P, b, c, c_out, omega, st, s);
}

hipError_t launch_q1_outer(int D, int prec, int n, int P, const void *c, double *R, double *U, const double *scal,
                           double f, double *part, hipStream_t st, void *cdefer, size_t cstride, double *adef,
                           const int *ctr, const Q1Shape &s) {
    const Q1Ring ring{cdefer, cstride, adef, ctr};
    if (cdefer) {
        if (!adef || !ctr) return hipErrorInvalidValue;
        Q1_DISPATCH(prec, TT, return (outer_t<TT, true>(D, n, P, c, R, U, scal, f, part, ring, s, st)));
    }
    Q1_DISPATCH(prec, TT, return (outer_t<TT, false>(D, n, P, c, R, U, scal, f, part, ring, s, st)));
}

hipError_t launch_q1_resid_flat(int D, int n, int P, const double *b, const double *U, double *R, double *uout,
                                double hd, double *part, hipStream_t st) {
    const unsigned N = npoints(D, n);
    const int blocks = flat_blocks((long)N);
    // r = b (no operator): the row-wise copy of the finite-difference path,
    // which writes the same flat_blocks(points) partials
    if (!U) return launch_resid_flat(D, n, P, b, nullptr, R, uout, 0.0, part, st);
    if (D == 3 && U && R && q1_final_lds_ok(n, P)) {
        // the LDS-staged form; it writes the partials of all `blocks`
        const Q1LdsShape s = q1_lds_shape(n, P, sizeof(double));
        hipLaunchKernelGGL((k_q1_lds<double, 3>), dim3(s.blocks), dim3((s.TY + 2) * (P / 4)), s.lds, st, b, U,
                           static_cast<void *>(uout), n, P, s.TY, s.zc, s.ytiles, 0.0, R, nullptr, nullptr, hd, part,
                           Q1Ring{}, blocks);
        return hipGetLastError();
    }
    if (D == 3)
        hipLaunchKernelGGL(k_q1_resid_flat<3>, dim3(blocks), dim3(kThreads), 0, st, b, U, R, uout, n, P, N, hd, part);
    else
        hipLaunchKernelGGL(k_q1_resid_flat<2>, dim3(blocks), dim3(kThreads), 0, st, b, U, R, uout, n, P, N, hd, part);
    return hipGetLastError();
}

hipError_t launch_q1_coarse(int D, int prec, const void *b, void *c, hipStream_t st) {
    Q1_DISPATCH(prec, TT, {
        if (D == 3)
            hipLaunchKernelGGL((k_q1_coarse<3, TT>), dim3(1), dim3(64), 0, st, static_cast<const TT *>(b),
                               static_cast<TT *>(c));
        else
            hipLaunchKernelGGL((k_q1_coarse<2, TT>), dim3(1), dim3(64), 0, st, static_cast<const TT *>(b),
                               static_cast<TT *>(c));
        return hipGetLastError();
    });
}

}  // namespace mg
