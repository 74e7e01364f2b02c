// gfx950 kernels for many right-hand sides sharing one 3-D operator, stored
// interleaved: the K values of a grid point are contiguous, element
// (x, y, z, k) at ((z*P + y)*P + x)*K + k of a padded level (pitch P, zero
// ghosts as in the single-grid layout).  Every right-hand side k goes through
// exactly the arithmetic of the single-grid kernels (same sum orders, same
// roundings), so column k of an interleaved solve reproduces a single-grid
// solve of that right-hand side; each column has its own scaling factor
// alpha_k and norms (Algorithm 2 per column), and columns whose flag act[k]
// is 0 are held fixed (their scaled right-hand side is zero and their update
// uses alpha = 0).
//
// Work decomposition: a thread owns V consecutive right-hand sides of one
// grid point of one row and marches along z, so a wave reads and writes
// contiguous runs of 64 V elements; x, y and z neighbours are whole V-chunks
// at offsets K, P K and P^2 K.
#include "mg_device.h"
#include "mg_launch.h"

#include <algorithm>
#include <type_traits>

namespace mg {
namespace {

struct MGrid {
    int P, K;
    __device__ __forceinline__ size_t at(int x, int y, int z) const {
        return (((size_t)z * P + (size_t)y) * P + (size_t)x) * K;
    }
    __device__ __forceinline__ bool interior(int x, int y, int z) const {
        return x >= 1 && x < P && y >= 1 && y < P && z >= 1 && z < P;
    }
};

// ---- fields: V values (right-hand sides k0 .. k0+V-1) at one grid point -----
template <class T, class A> struct MArr {
    typedef A acc;
    const T *__restrict__ p;
    template <int V> __device__ __forceinline__ void get(const MGrid &g, int x, int y, int z, int k0, A (&o)[V]) const {
        if (!g.interior(x, y, z)) {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = A(0);
            return;
        }
        load_row<T, V>(p + g.at(x, y, z) + k0, o);
    }
};

// round_T(r_k / alpha_k) of the FP64 residual, zero for held columns.
template <class T, int V> struct MScaled {
    typedef acc_t<T> acc;
    const double *__restrict__ r;
    double inv[V];
    bool on[V];
    template <int W> __device__ __forceinline__ void get(const MGrid &g, int x, int y, int z, int k0, acc (&o)[W]) const {
        static_assert(W == V, "one chunk width per kernel");
        if (!g.interior(x, y, z)) {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = acc(0);
            return;
        }
        double rv[V];
        load_row<double, V>(r + g.at(x, y, z) + k0, rv);
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = on[i] ? widen(Store<T>::from_f64(rv[i] * inv[i])) : acc(0);
    }
};

// First Jacobi iterate from zero: round_T(k b).
template <class T, class R> struct MJac0 {
    typedef acc_t<T> acc;
    R rhs;
    acc k;
    template <int V> __device__ __forceinline__ void get(const MGrid &g, int x, int y, int z, int k0, acc (&o)[V]) const {
        rhs.template get<V>(g, x, y, z, k0, o);
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = round_to<T>(k * o[i]);
    }
};

// round_TF(c + 4 P e_c) with the interpolation sums in the canonical order of
// the single-grid kernels: per contributing coarse row, the z sum over
// interior coarse planes, then the y weights, then the x weights.
template <class TF, class TC> struct MProl {
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

    template <int V> __device__ __forceinline__ void colsum(int K, int X, int y, int z, int k0, PA (&s)[V]) const {
        const MGrid gc{Pc, K};
#pragma unroll
        for (int i = 0; i < V; ++i) s[i] = PA(0);
        int Zs[2], Ys[2];
        const int nz = split(z, Zs), ny = split(y, Ys);
        const PA wz = nz == 1 ? PA(1) : PA(0.5), wy = ny == 1 ? PA(1) : PA(0.5);
        for (int bb = 0; bb < ny; ++bb) {
            const int Y = Ys[bb];
            PA t[V];
#pragma unroll
            for (int i = 0; i < V; ++i) t[i] = PA(0);
            if (X >= 1 && X < Pc && Y >= 1 && Y < Pc) {
                for (int a = 0; a < nz; ++a) {
                    const int Z = Zs[a];
                    if (Z < 1 || Z >= Pc) continue;
                    PA v[V];
                    load_row<TC, V>(ec + gc.at(X, Y, Z) + k0, v);
#pragma unroll
                    for (int i = 0; i < V; ++i) t[i] += wz * v[i];
                }
            }
#pragma unroll
            for (int i = 0; i < V; ++i) s[i] += wy * t[i];
        }
    }

    template <int V> __device__ __forceinline__ void get(const MGrid &g, int x, int y, int z, int k0, acc (&o)[V]) const {
        if (!g.interior(x, y, z)) {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = acc(0);
            return;
        }
        PA p[V];
        if ((x & 1) == 0) {
            colsum<V>(g.K, x >> 1, y, z, k0, p);
        } else {
            PA s1[V];
            colsum<V>(g.K, (x - 1) >> 1, y, z, k0, p);
            colsum<V>(g.K, (x + 1) >> 1, y, z, k0, s1);
#pragma unroll
            for (int i = 0; i < V; ++i) p[i] = PA(0.5) * (p[i] + s1[i]);
        }
        acc cv[V];
        load_row<TF, V>(c + g.at(x, y, z) + k0, cv);
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = round_to<TF>((PA)cv[i] + PA(4) * p[i]);
    }
};

// ---- emit policies ----------------------------------------------------------
template <class T, class R, bool WRITE_B> struct MSweep {
    typedef acc_t<T> A;
    R rhs;
    T *__restrict__ out;
    T *__restrict__ bout;
    A k;
    template <int V>
    __device__ __forceinline__ void emit(const MGrid &g, int x, int y, int z, int k0, const A (&c)[V],
                                         const A (&nb)[V]) {
        A b[V];
        rhs.template get<V>(g, x, y, z, k0, b);
        T o[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const A lc = fmaT<A>(A(6), c[i], -nb[i]);
            o[i] = Store<T>::from_acc(fmaT<A>(k, b[i] - lc, c[i]));
        }
        const size_t at = g.at(x, y, z) + k0;
        store_row<T, V>(out + at, o);
        if (WRITE_B) {
            T bo[V];
#pragma unroll
            for (int i = 0; i < V; ++i) bo[i] = Store<T>::from_acc(b[i]);
            store_row<T, V>(bout + at, bo);
        }
    }
};

// Refinement update per column: u += a_k h^2 c, r -= a_k (6 c - nb), with
// a_k = alpha_k for stepping columns and 0 for held ones; per-column
// (sum r^2, max |r|) partials.
template <int V> struct MOuter {
    typedef double A;
    double *__restrict__ R;
    double *__restrict__ U;
    double a[V];
    double h2;
    double *__restrict__ part;
    double ss[V], mx[V];
    template <int W>
    __device__ __forceinline__ void emit(const MGrid &g, int x, int y, int z, int k0, const A (&c)[W],
                                         const A (&nb)[W]) {
        static_assert(W == V, "one chunk width per kernel");
        const size_t at = g.at(x, y, z) + k0;
        double r[V], u[V];
        load_row<double, V>(R + at, r);
        load_row<double, V>(U + at, u);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const double ah2 = a[i] * h2;
            const double lc = fmaT<double>(6.0, c[i], -nb[i]);
            r[i] = fmaT<double>(-a[i], lc, r[i]);
            u[i] = fmaT<double>(ah2, c[i], u[i]);
            ss[i] += r[i] * r[i];
            mx[i] = nanmax(mx[i], fabs(r[i]));
        }
        store_row<double, V>(R + at, r);
        store_row<double, V>(U + at, u);
    }
    __device__ __forceinline__ void finish(double *lds, int K, int kc, long blk);
};

// Per-column block reduction.  Thread t holds V columns k0 = (t mod KC) V ..;
// lanes that agree modulo KC combine with an xor butterfly, then the waves in
// order through LDS (8 K doubles).  Writes part[(blk K + k) 2 + {0, 1}].
template <int V>
__device__ __forceinline__ void reduce_columns(double (&ss)[V], double (&mx)[V], double *lds, int K, int kc,
                                               double *part, long blk) {
    const int KC = K / V;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        for (int off = KC; off < 64; off <<= 1) {
            ss[i] += __shfl_xor(ss[i], off, 64);
            mx[i] = nanmax(mx[i], __shfl_xor(mx[i], off, 64));
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane < KC) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
            lds[(w * K + kc * V + i) * 2] = ss[i];
            lds[(w * K + kc * V + i) * 2 + 1] = mx[i];
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
        const int k = threadIdx.x;
        double s = 0.0, m = 0.0;
        for (int q = 0; q < nw; ++q) {
            s += lds[(q * K + k) * 2];
            m = nanmax(m, lds[(q * K + k) * 2 + 1]);
        }
        part[(blk * K + k) * 2] = s;
        part[(blk * K + k) * 2 + 1] = m;
    }
}

template <int V> __device__ __forceinline__ void MOuter<V>::finish(double *lds, int K, int kc, long blk) {
    reduce_columns<V>(ss, mx, lds, K, kc, part, blk);
}

// ---- the z-marching stencil ----------------------------------------------------
// Thread t: chunk xk = t mod TXR of row line = t div TXR, TXR = (P-1) K/V
// (interior points only: ghost points are never written and stay zero).
struct MMap {
    int x, y, kc, k0, z0, z1;
    bool active;
};

template <int V> __device__ __forceinline__ MMap mmap(int P, int K, int zc, int nchunks) {
    const int KC = K / V;
    const long TXR = (long)(P - 1) * KC;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long xk = t % TXR, line = t / TXR;
    MMap m;
    m.x = 1 + (int)(xk / KC);
    m.kc = (int)(xk % KC);
    m.k0 = m.kc * V;
    m.y = 1 + (int)(line % (P - 1));
    const int chunk = (int)(line / (P - 1));
    m.active = chunk < nchunks;
    m.z0 = 1 + chunk * zc;
    m.z1 = min(m.z0 + zc, P);
    return m;
}

// Row-segment decomposition of the stencil kernels: a workgroup owns up to
// segx consecutive interior points of one row (all K columns) and a chunk of
// planes; thread t holds columns (t mod KC) V .. of point xs + t div KC.  The
// plane being swept passes through LDS (two slots), so the x neighbours come
// from the neighbouring threads (from memory only at the segment ends): three
// field reads per point and plane instead of five.  The thread count is
// rounded up to whole waves (the spare threads compute nothing that is kept).
struct MSeg {
    int segx, nseg, threads;
};
__host__ __device__ inline MSeg mseg_shape(int V, int P, int K, int maxthr = 1024) {
    const int KC = K / V;
    MSeg s;
    s.segx = (P - 1) < maxthr / KC ? (P - 1) : maxthr / KC;
    s.nseg = (P - 1 + s.segx - 1) / s.segx;
    s.threads = (s.segx * KC + 63) / 64 * 64;
    return s;
}

struct MSegMap {
    int x, y, kc, k0, z0, z1, xs, xe;
    bool run;  // the workgroup has planes to do (uniform)
    bool own;  // the thread's point is one of the segment's
};

template <int V> __device__ __forceinline__ MSegMap msegmap(int P, int K, int zc, int nchunks, int maxthr = 1024) {
    const int KC = K / V;
    const MSeg s = mseg_shape(V, P, K, maxthr);
    const int seg = (int)(blockIdx.x % s.nseg);
    const long rest = blockIdx.x / s.nseg;
    MSegMap m;
    m.xs = 1 + seg * s.segx;
    m.xe = min(P - 1, m.xs + s.segx - 1);
    m.x = m.xs + (int)threadIdx.x / KC;
    m.kc = (int)threadIdx.x % KC;
    m.k0 = m.kc * V;
    m.y = 1 + (int)(rest % (P - 1));
    const int chunk = (int)(rest / (P - 1));
    m.run = chunk < nchunks;
    m.own = m.x <= m.xe;
    m.z0 = 1 + chunk * zc;
    m.z1 = min(m.z0 + zc, P);
    return m;
}

template <int V, class F, class E>
__device__ __forceinline__ void mstencil_seg_body(const F &f, E &e, const MGrid &g, const MSegMap &m,
                                                  typename F::acc *lds) {
    typedef typename F::acc A;
    const int KC = g.K / V;
    const int t = threadIdx.x;
    const size_t slot = (size_t)blockDim.x * V;
    A cm[V], cc[V], cp[V];
    f.template get<V>(g, m.x, m.y, m.z0 - 1, m.k0, cm);
    f.template get<V>(g, m.x, m.y, m.z0, m.k0, cc);
    store_row<A, V>(lds + (size_t)t * V, cc);
    __syncthreads();
    for (int z = m.z0; z < m.z1; ++z) {
        const int it = z - m.z0;
        f.template get<V>(g, m.x, m.y, z + 1, m.k0, cp);
        const A *row = lds + (size_t)(it & 1) * slot;
        A xl[V], xr[V], ym[V], yp[V], nb[V];
        if (m.x > m.xs)
            load_row<A, V>(row + (size_t)(t - KC) * V, xl);
        else
            f.template get<V>(g, m.x - 1, m.y, z, m.k0, xl);
        if (m.x < m.xe)
            load_row<A, V>(row + (size_t)(t + KC) * V, xr);
        else
            f.template get<V>(g, m.x + 1, m.y, z, m.k0, xr);
        f.template get<V>(g, m.x, m.y - 1, z, m.k0, ym);
        f.template get<V>(g, m.x, m.y + 1, z, m.k0, yp);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            nb[i] = xl[i] + xr[i];
            nb[i] += ym[i];
            nb[i] += yp[i];
            nb[i] += cm[i];
            nb[i] += cp[i];
        }
        if (m.own) e.template emit<V>(g, m.x, m.y, z, m.k0, cc, nb);
        // plane z+1 into the other slot: it was last read before the previous barrier
        store_row<A, V>(lds + (size_t)((it + 1) & 1) * slot + (size_t)t * V, cp);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < V; ++i) {
            cm[i] = cc[i];
            cc[i] = cp[i];
        }
    }
}

template <int V, class F, class E>
__device__ __forceinline__ void mstencil_body(const F &f, E &e, const MGrid &g, const MMap &m) {
    typedef typename F::acc A;
    if (!m.active) return;
    A cm[V], cc[V], cp[V];
    f.template get<V>(g, m.x, m.y, m.z0 - 1, m.k0, cm);
    f.template get<V>(g, m.x, m.y, m.z0, m.k0, cc);
    for (int z = m.z0; z < m.z1; ++z) {
        f.template get<V>(g, m.x, m.y, z + 1, m.k0, cp);
        A xl[V], xr[V], ym[V], yp[V], nb[V];
        f.template get<V>(g, m.x - 1, m.y, z, m.k0, xl);
        f.template get<V>(g, m.x + 1, m.y, z, m.k0, xr);
        f.template get<V>(g, m.x, m.y - 1, z, m.k0, ym);
        f.template get<V>(g, m.x, m.y + 1, z, m.k0, yp);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            nb[i] = xl[i] + xr[i];
            nb[i] += ym[i];
            nb[i] += yp[i];
            nb[i] += cm[i];
            nb[i] += cp[i];
        }
        e.template emit<V>(g, m.x, m.y, z, m.k0, cc, nb);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            cm[i] = cc[i];
            cc[i] = cp[i];
        }
    }
}

enum { MK_SMOOTH2 = 0, MK_SMOOTH2_SCALED = 1, MK_SWEEP = 2 };

template <int V, int KIND, class T, class TC>
__global__ __launch_bounds__(1024) void k_mstencil(const void *b, const double *r, const double *inv, const int *act,
                                                   void *bout, const void *cin, const void *ec, void *cout, int P,
                                                   int K, int zc, int nchunks, double omega) {
    typedef acc_t<T> A;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A *lds = reinterpret_cast<A *>(smem_raw);
    const MGrid g{P, K};
    const MSegMap m = msegmap<V>(P, K, zc, nchunks);
    if (!m.run) return;
    const A kw = (A)(omega / 6.0);
    if constexpr (KIND == MK_SMOOTH2) {
        typedef MArr<T, A> R;
        const R rh{static_cast<const T *>(b)};
        const MJac0<T, R> f{rh, kw};
        MSweep<T, R, false> e{rh, static_cast<T *>(cout), nullptr, kw};
        mstencil_seg_body<V>(f, e, g, m, lds);
    } else if constexpr (KIND == MK_SMOOTH2_SCALED) {
        typedef MScaled<T, V> R;
        R rh;
        rh.r = r;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            rh.inv[i] = inv[m.k0 + i];
            rh.on[i] = act[m.k0 + i] != 0;
        }
        const MJac0<T, R> f{rh, kw};
        MSweep<T, R, true> e{rh, static_cast<T *>(cout), static_cast<T *>(bout), kw};
        mstencil_seg_body<V>(f, e, g, m, lds);
    } else {
        typedef MArr<T, A> R;
        const R f{static_cast<const T *>(cin)};
        MSweep<T, R, false> e{R{static_cast<const T *>(b)}, static_cast<T *>(cout), nullptr, kw};
        mstencil_seg_body<V>(f, e, g, m, lds);
    }
}

// The update holds its field and R, U in FP64: 4 columns per thread in every
// format, at most 512 threads, so that its registers need not spill.
constexpr int kUpdThreads = 512;
constexpr int kUpdVec = 4;

template <int V, class T>
__global__ __launch_bounds__(kUpdThreads) void k_mupdate(const T *c, double *R, double *U, const double *alpha,
                                                         const int *act, double h2, double *part, int P, int K,
                                                         int zc, int nchunks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);  // the plane slots, then the column reduction
    const MGrid g{P, K};
    const MSegMap m = msegmap<V>(P, K, zc, nchunks, kUpdThreads);
    const MArr<T, double> f{c};
    MOuter<V> e;
    e.R = R, e.U = U, e.h2 = h2, e.part = part;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        e.a[i] = act[m.k0 + i] ? alpha[m.k0 + i] : 0.0;
        e.ss[i] = 0.0, e.mx[i] = 0.0;
    }
    if (m.run) mstencil_seg_body<V>(f, e, g, m, lds);
    e.finish(lds, K, m.kc, blockIdx.x);
}

// ---- two-pass residual + restriction and prolongation -------------------------
// Pass 1 stores the fine residual b - (6 c - nb) in the fine accumulator type
// (the exact value the fused form keeps in registers); pass 2 applies the
// full-weighting weights in the fused form's order.  The prolongation first
// replaces c by round(c + 4 P e) in place (every point reads only its own c),
// then a plain sweep runs on it.  Same results as the fused kernels, with
// every pass a streaming one.
template <class TF, class A> struct MResidOut {
    const TF *__restrict__ b;
    A *__restrict__ r;
    template <int V>
    __device__ __forceinline__ void emit(const MGrid &g, int x, int y, int z, int k0, const A (&c)[V],
                                         const A (&nb)[V]) {
        A bb[V], rv[V];
        load_row<TF, V>(b + g.at(x, y, z) + k0, bb);
#pragma unroll
        for (int i = 0; i < V; ++i) rv[i] = bb[i] - fmaT<A>(A(6), c[i], -nb[i]);
        store_row<A, V>(r + g.at(x, y, z) + k0, rv);
    }
};

template <int V, class TF>
__global__ __launch_bounds__(1024) void k_mresid_store(const TF *b, const TF *c, acc_t<TF> *r, int P, int K, int zc,
                                                       int nchunks) {
    typedef acc_t<TF> A;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const MGrid g{P, K};
    const MSegMap m = msegmap<V>(P, K, zc, nchunks);
    if (!m.run) return;
    const MArr<TF, A> f{c};
    MResidOut<TF, A> e{b, r};
    mstencil_seg_body<V>(f, e, g, m, reinterpret_cast<A *>(smem_raw));
}

// Coarse point (X, Y) and V columns, marching over coarse planes; reads the
// stored fine residuals of the 3 x 3 fine points under (X, Y) per fine plane.
template <int V, class A, class TC>
__global__ __launch_bounds__(256) void k_mfw(const A *r, TC *bc, int P, int K, int zcc, int nzch) {
    const int Pc = P >> 1, KC = K / V;
    const MGrid g{P, K}, gc{Pc, K};
    const long TXC = (long)(Pc - 1) * KC;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long xk = t % TXC, line = t / TXC;
    const int X = 1 + (int)(xk / KC), k0 = (int)(xk % KC) * V;
    const int Y = 1 + (int)(line % (Pc - 1));
    const int zch = (int)(line / (Pc - 1));
    if (zch >= nzch) return;
    const int Z0 = 1 + zch * zcc, Z1 = min(Z0 + zcc, Pc);
    const int zf0 = 2 * Z0 - 1, zf1 = 2 * Z1 - 1;
    A acc[V];
    for (int zf = zf0; zf <= zf1; ++zf) {
        A rs[3][V];
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            A r0[V], r1[V], r2[V];
            const size_t base = g.at(2 * X - 1, 2 * Y - 1 + oy, zf) + k0;
            load_row<A, V>(r + base, r0);
            load_row<A, V>(r + base + K, r1);
            load_row<A, V>(r + base + 2 * (size_t)K, r2);
#pragma unroll
            for (int i = 0; i < V; ++i) rs[oy][i] = A(0.25) * (r0[i] + r2[i]) + A(0.5) * r1[i];
        }
        A q[V];
#pragma unroll
        for (int i = 0; i < V; ++i) q[i] = A(0.25) * (rs[0][i] + rs[2][i]) + A(0.5) * rs[1][i];
        if (zf == zf0) {
#pragma unroll
            for (int i = 0; i < V; ++i) acc[i] = A(0.25) * q[i];
        } else if (((zf - zf0) & 1) == 1) {
#pragma unroll
            for (int i = 0; i < V; ++i) acc[i] += A(0.5) * q[i];
        } else {
            TC out[V];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                out[i] = store_as<TC>(acc[i] + A(0.25) * q[i]);
                acc[i] = A(0.25) * q[i];
            }
            store_row<TC, V>(bc + gc.at(X, Y, (zf - 1) >> 1) + k0, out);
        }
    }
}

// c = round_TF(c + 4 P e_c) in place at every interior point.
template <int V, class TF, class TC>
__global__ __launch_bounds__(256) void k_mprol_field(TF *c, const TC *ec, int P, int K, int zc, int nchunks) {
    typedef MProl<TF, TC> F;
    typedef typename F::PA PA;
    const MGrid g{P, K};
    const MMap m = mmap<V>(P, K, zc, nchunks);
    if (!m.active) return;
    // The coarse values of the (up to) 2 x 2 coarse columns around (x, y) are
    // loaded once per coarse plane and kept for the two or three fine planes
    // that use it (slot Z & 1), instead of once per fine plane; the sums are
    // those of MProl::get, in its order.
    const int Pc = P / 2;
    const MGrid gc{Pc, K};
    int Xs[2] = {0, 0}, Ys[2] = {0, 0};
    const int nx = F::split(m.x, Xs), ny = F::split(m.y, Ys);
    const PA wy = ny == 1 ? PA(1) : PA(0.5);
    PA ce[2][2][V], co[2][2][V];  // coarse planes of even and of odd index
    int tag_e = -1, tag_o = -1;
    auto load_plane = [&](int Z, PA (&dst)[2][2][V]) {
#pragma unroll
        for (int bx = 0; bx < 2; ++bx)
#pragma unroll
            for (int by = 0; by < 2; ++by)
                if (bx < nx && by < ny && Xs[bx] >= 1 && Xs[bx] < Pc && Ys[by] >= 1 && Ys[by] < Pc)
                    load_row<TC, V>(ec + gc.at(Xs[bx], Ys[by], Z) + m.k0, dst[bx][by]);
    };
    for (int z = m.z0; z < m.z1; ++z) {
        int Zs[2] = {0, 0};
        const int nz = F::split(z, Zs);
        const PA wz = nz == 1 ? PA(1) : PA(0.5);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (a >= nz) break;
            const int Z = Zs[a];
            if (Z < 1 || Z >= Pc) continue;
            if (Z & 1) {
                if (tag_o != Z) load_plane(Z, co), tag_o = Z;
            } else {
                if (tag_e != Z) load_plane(Z, ce), tag_e = Z;
            }
        }
        PA p[V];
#pragma unroll
        for (int bx = 0; bx < 2; ++bx) {
            if (bx >= nx) break;
            PA s[V];
#pragma unroll
            for (int i = 0; i < V; ++i) s[i] = PA(0);
#pragma unroll
            for (int by = 0; by < 2; ++by) {
                if (by >= ny) break;
                PA t[V];
#pragma unroll
                for (int i = 0; i < V; ++i) t[i] = PA(0);
                if (Xs[bx] >= 1 && Xs[bx] < Pc && Ys[by] >= 1 && Ys[by] < Pc) {
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        if (a >= nz) break;
                        const int Z = Zs[a];
                        if (Z < 1 || Z >= Pc) continue;
                        if (Z & 1) {
#pragma unroll
                            for (int i = 0; i < V; ++i) t[i] += wz * co[bx][by][i];
                        } else {
#pragma unroll
                            for (int i = 0; i < V; ++i) t[i] += wz * ce[bx][by][i];
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < V; ++i) s[i] += wy * t[i];
            }
            if (bx == 0) {
#pragma unroll
                for (int i = 0; i < V; ++i) p[i] = s[i];
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) p[i] = PA(0.5) * (p[i] + s[i]);
            }
        }
        acc_t<TF> cv[V];
        load_row<TF, V>(c + g.at(m.x, m.y, z) + m.k0, cv);
        TF o[V];
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = Store<TF>::from_acc(round_to<TF>((PA)cv[i] + PA(4) * p[i]));
        store_row<TF, V>(c + g.at(m.x, m.y, z) + m.k0, o);
    }
}

// Base level (n = 1): c = b / 6 at the single interior point, every column.
template <class T> __global__ void k_mcoarse(const T *b, T *c, int K) {
    const int k = threadIdx.x;
    if (k >= K) return;
    typedef acc_t<T> A;
    const size_t at = (size_t)7 * K + k;
    c[at] = Store<T>::from_acc(widen(b[at]) / A(6));
}

// r = b - A U (or r = b when U is null) for the columns with mask[k] != 0:
// one wave per grid row, lane l always on column l mod K (K divides 64), so
// the per-column partials need no index arithmetic.  Optionally stores R and
// copies U out to the dense uout (all columns).
__global__ __launch_bounds__(256) void k_mresid(const double *__restrict__ b, const double *__restrict__ U,
                                                double *__restrict__ R, double *__restrict__ uout,
                                                const int *__restrict__ mask, int n, int P, int K, double inv_h2,
                                                double *__restrict__ part) {
    __shared__ double lds[8 * 64];
    const MGrid g{P, K};
    const size_t xs = (size_t)K, ys = (size_t)P * K, zs = (size_t)P * P * K;
    const long rows = (long)n * n;
    const long rowlen = (long)n * K;
    const int lane = threadIdx.x & 63;
    const int kl = lane % K;
    const bool on = mask == nullptr || mask[kl] != 0;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    double ss[1] = {0.0}, mx[1] = {0.0};
    for (long row = wave; row < rows; row += nwaves) {
        const int y = (int)(row % n) + 1, z = (int)(row / n) + 1;
        const size_t dbase = (size_t)row * rowlen;
        const size_t pbase = g.at(1, y, z);
        for (long e = lane; e < rowlen; e += 64) {
            const size_t p = pbase + e;
            if (uout) uout[dbase + e] = U[p];
            if (!on) continue;
            double r = b[dbase + e];
            if (U) {
                double nb = U[p - xs] + U[p + xs];
                nb += U[p - ys];
                nb += U[p + ys];
                nb += U[p - zs];
                nb += U[p + zs];
                r = r - (6.0 * U[p] - nb) * inv_h2;
            }
            if (R) R[p] = r;
            ss[0] += r * r;
            mx[0] = nanmax(mx[0], fabs(r));
        }
    }
    // lanes equal modulo K hold the same column: reduce_columns with V = 1
    reduce_columns<1>(ss, mx, lds, K, kl, part, blockIdx.x);
}

// Dense interleaved n^3 K -> padded interior (other entries untouched);
// columns with keep[k] == 0 are written as zeros.
__global__ __launch_bounds__(256) void k_mpack(const double *__restrict__ src, double *__restrict__ dst, int n, int P,
                                               int K, const int *__restrict__ keep) {
    const MGrid g{P, K};
    const long rows = (long)n * n, rowlen = (long)n * K;
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    for (long row = wave; row < rows; row += nwaves) {
        const int y = (int)(row % n) + 1, z = (int)(row / n) + 1;
        for (long e = lane; e < rowlen; e += 64)
            dst[g.at(1, y, z) + e] = keep[lane % K] ? src[(size_t)row * rowlen + e] : 0.0;
    }
}

// Per-column reduction of the partials (one block per column k with
// mask[k] != 0): scal = {alpha[K], 1/alpha[K], ||r||_2[K], ||r||_inf[K]}.
__global__ __launch_bounds__(256) void k_mfinalize(const double *__restrict__ part, int nparts, int K,
                                                   double *__restrict__ scal, const int *__restrict__ mask,
                                                   int scaling) {
    __shared__ double red[8];
    const int k = blockIdx.x;
    if (mask && !mask[k]) return;
    double s = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        s += part[((size_t)i * K + k) * 2];
        m = nanmax(m, part[((size_t)i * K + k) * 2 + 1]);
    }
    block_reduce(s, m, red);
    if (threadIdx.x == 0) {
        double a = scaling ? ldexp(m, scaling - 1) : 1.0;
        if (!(a > 0.0) || a > 1.7e308) a = 1.0;
        scal[k] = a;
        scal[K + k] = 1.0 / a;
        scal[2 * K + k] = sqrt(s);
        scal[3 * K + k] = m;
    }
}

int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

#define MG_MT(prec, ...)                                   \
    switch (prec) {                                        \
    case P_F64: { typedef double TT; __VA_ARGS__; break; } \
    case P_F32: { typedef float TT; __VA_ARGS__; break; }  \
    case P_F16: { typedef f16 TT; __VA_ARGS__; break; }    \
    case P_BF16: { typedef bf16 TT; __VA_ARGS__; break; }  \
    default: return hipErrorInvalidValue;                  \
    }

// LDS of a row-segment kernel: two plane slots of V accumulator values per
// thread (and room for the update's per-column reduction).
size_t mseg_lds(int V, size_t acc, const MSeg &s, int K) {
    return std::max((size_t)2 * s.threads * V * acc, (size_t)2 * (s.threads / 64) * K * sizeof(double));
}

// Workgroups of the pointwise prolongation (256 threads, thread t as in mmap).
int m_flat_blocks(int prec, int P, int K, int zc) {
    const long threads = (long)(P - 1) * (K / m_vec(prec)) * (P - 1) * cdiv(P - 1, zc);
    return cdiv(threads, 256);
}

template <int KIND, class T, class TC>
hipError_t mstencil_run(const MArgs &a, hipStream_t st) {
    constexpr int V = std::is_same<T, double>::value ? 4 : 8;
    const int nch = cdiv(a.P - 1, a.zc);
    const int blocks = m_stencil_blocks(a.prec, a.P, a.K, a.zc);
    const MSeg sg = mseg_shape(V, a.P, a.K);
    hipLaunchKernelGGL((k_mstencil<V, KIND, T, TC>), dim3(blocks), dim3(sg.threads),
                       mseg_lds(V, sizeof(acc_t<T>), sg, a.K), st, a.b, a.r, a.inv, a.act, a.bout, a.cin, a.ec,
                       a.cout, a.P, a.K, a.zc, nch, a.omega);
    return hipGetLastError();
}

template <int KIND, class T> hipError_t mstencil_tc(const MArgs &a, hipStream_t st) {
    return mstencil_run<KIND, T, double>(a, st);
}

template <int KIND> hipError_t mstencil_kind(const MArgs &a, hipStream_t st) {
    MG_MT(a.prec, return mstencil_tc<KIND, TT>(a, st));
    return hipErrorInvalidValue;
}

template <class TF> hipError_t mresid_store_run(const MArgs &a, void *rbuf, hipStream_t st) {
    constexpr int V = std::is_same<TF, double>::value ? 4 : 8;
    const int nch = cdiv(a.P - 1, a.zc);
    const int blocks = m_stencil_blocks(a.prec, a.P, a.K, a.zc);
    const MSeg sg = mseg_shape(V, a.P, a.K);
    hipLaunchKernelGGL((k_mresid_store<V, TF>), dim3(blocks), dim3(sg.threads),
                       mseg_lds(V, sizeof(acc_t<TF>), sg, a.K), st, static_cast<const TF *>(a.b),
                       static_cast<const TF *>(a.cin), static_cast<acc_t<TF> *>(rbuf), a.P, a.K, a.zc, nch);
    return hipGetLastError();
}

template <class TF, class TC> hipError_t mfw_run(const MArgs &a, const void *rbuf, int zcc, hipStream_t st) {
    constexpr int V = std::is_same<TF, double>::value ? 4 : 8;
    const int Pc = a.P / 2;
    const int nz = cdiv(Pc - 1, zcc);
    const long threads = (long)(Pc - 1) * (a.K / V) * (Pc - 1) * nz;
    hipLaunchKernelGGL((k_mfw<V, acc_t<TF>, TC>), dim3(cdiv(threads, 256)), dim3(256), 0, st,
                       static_cast<const acc_t<TF> *>(rbuf), static_cast<TC *>(a.cout), a.P, a.K, zcc, nz);
    return hipGetLastError();
}

template <class TF, class TC> hipError_t mprol_field_run(const MArgs &a, hipStream_t st) {
    constexpr int V = std::is_same<TF, double>::value ? 4 : 8;
    const int nch = cdiv(a.P - 1, a.zc);
    const int blocks = m_flat_blocks(a.prec, a.P, a.K, a.zc);
    hipLaunchKernelGGL((k_mprol_field<V, TF, TC>), dim3(blocks), dim3(256), 0, st,
                       static_cast<TF *>(const_cast<void *>(a.cin)), static_cast<const TC *>(a.ec), a.P, a.K, a.zc,
                       nch);
    return hipGetLastError();
}

}  // namespace

int m_vec(int prec) { return prec == P_F64 ? 4 : 8; }

bool m_supported(int prec, int K) {
    const int V = m_vec(prec);
    return K >= V && K <= 64 && (K & (K - 1)) == 0;
}

int m_stencil_blocks(int prec, int P, int K, int zc) {
    return mseg_shape(m_vec(prec), P, K).nseg * (P - 1) * cdiv(P - 1, zc);
}

int m_update_blocks(int, int P, int K, int zc) {
    return mseg_shape(kUpdVec, P, K, kUpdThreads).nseg * (P - 1) * cdiv(P - 1, zc);
}

int m_resid_blocks(int n) { return std::max(1, std::min(cdiv((long)n * n, 4), 4096)); }

hipError_t launch_m_stage(int kind, const MArgs &a, hipStream_t st) {
    if (!m_supported(a.prec, a.K) || a.P < 4 || a.zc < 1) return hipErrorInvalidValue;
    switch (kind) {
    case MS_SMOOTH2: return a.r ? mstencil_kind<MK_SMOOTH2_SCALED>(a, st) : mstencil_kind<MK_SMOOTH2>(a, st);
    case MS_SWEEP: return mstencil_kind<MK_SWEEP>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_m_update(const MArgs &a, double *R, double *U, const double *alpha, double h2, double *part,
                           hipStream_t st) {
    if (!m_supported(a.prec, a.K)) return hipErrorInvalidValue;
    const int nch = cdiv(a.P - 1, a.zc);
    const int blocks = m_update_blocks(a.prec, a.P, a.K, a.zc);
    MG_MT(a.prec, {
        constexpr int V = kUpdVec;
        const MSeg sg = mseg_shape(V, a.P, a.K, kUpdThreads);
        hipLaunchKernelGGL((k_mupdate<V, TT>), dim3(blocks), dim3(sg.threads), mseg_lds(V, sizeof(double), sg, a.K),
                           st, static_cast<const TT *>(a.cin), R, U, alpha, a.act, h2, part, a.P, a.K, a.zc, nch);
    });
    return hipGetLastError();
}

hipError_t launch_m_coarse(int prec, int K, const void *b, void *c, hipStream_t st) {
    MG_MT(prec, hipLaunchKernelGGL((k_mcoarse<TT>), dim3(1), dim3(64), 0, st, static_cast<const TT *>(b),
                                   static_cast<TT *>(c), K));
    return hipGetLastError();
}

hipError_t launch_m_resid(int n, int P, int K, const double *b, const double *U, double *R, double *uout,
                          const int *mask, double inv_h2, double *part, hipStream_t st) {
    if (K < 1 || K > 64 || (K & (K - 1))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mresid, dim3(m_resid_blocks(n)), dim3(256), 0, st, b, U, R, uout, mask, n, P, K, inv_h2,
                       part);
    return hipGetLastError();
}

hipError_t launch_m_pack(int n, int P, int K, const double *src, double *dst, const int *keep, hipStream_t st) {
    if (K < 1 || K > 64 || (K & (K - 1))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mpack, dim3(m_resid_blocks(n)), dim3(256), 0, st, src, dst, n, P, K, keep);
    return hipGetLastError();
}

hipError_t launch_m_finalize(const double *part, int nparts, int K, double *scal, const int *mask, int scaling,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_mfinalize, dim3(K), dim3(256), 0, st, part, nparts, K, scal, mask, scaling);
    return hipGetLastError();
}

size_t m_resid_bytes(int prec, size_t elems) { return elems * (prec == P_F64 ? 8 : 4); }

hipError_t launch_m_restrict2(const MArgs &a, void *rbuf, int zcc, hipStream_t st) {
    if (!m_supported(a.prec, a.K) || a.P < 4 || a.zc < 1 || zcc < 1) return hipErrorInvalidValue;
    hipError_t e = hipErrorInvalidValue;
    MG_MT(a.prec, e = mresid_store_run<TT>(a, rbuf, st));
    if (e != hipSuccess) return e;
    switch (a.prec) {
    case P_F64: MG_MT(a.pc, return (mfw_run<double, TT>(a, rbuf, zcc, st))); break;
    case P_F32: MG_MT(a.pc, return (mfw_run<float, TT>(a, rbuf, zcc, st))); break;
    case P_F16: MG_MT(a.pc, return (mfw_run<f16, TT>(a, rbuf, zcc, st))); break;
    case P_BF16: MG_MT(a.pc, return (mfw_run<bf16, TT>(a, rbuf, zcc, st))); break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_m_prolong_field(const MArgs &a, hipStream_t st) {
    if (!m_supported(a.prec, a.K) || a.P < 4 || a.zc < 1) return hipErrorInvalidValue;
    switch (a.prec) {
    case P_F64: MG_MT(a.pc, return (mprol_field_run<double, TT>(a, st))); break;
    case P_F32: MG_MT(a.pc, return (mprol_field_run<float, TT>(a, st))); break;
    case P_F16: MG_MT(a.pc, return (mprol_field_run<f16, TT>(a, st))); break;
    case P_BF16: MG_MT(a.pc, return (mprol_field_run<bf16, TT>(a, st))); break;
    }
    return hipErrorInvalidValue;
}

}  // namespace mg
