// Device-side building blocks of the gfx950 multigrid kernels: storage
// formats and their rounding, vector row loads/stores, the padded level
// layout, and wave64 reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mg {

// ---------------------------------------------------------------------------
// Storage formats.  FP16 uses the compiler's _Float16; BF16 is stored as its
// 16-bit pattern and converted by hand (exact widening, RNE narrowing).
struct bf16 {
    uint16_t u;
};
typedef _Float16 f16;

template <class T> struct acc_of { typedef float type; };
template <> struct acc_of<double> { typedef double type; };
template <class T> using acc_t = typename acc_of<T>::type;

__device__ __forceinline__ float widen(f16 v) { return (float)v; }
__device__ __forceinline__ float widen(bf16 v) { return __uint_as_float((uint32_t)v.u << 16); }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ double widen(double v) { return v; }

// float -> bf16, round to nearest even (integer bias method); NaN stays NaN.
__device__ __forceinline__ bf16 f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    bf16 r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        r.u = (uint16_t)((u >> 16) | 0x40u);
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);
        r.u = (uint16_t)(u >> 16);
    }
    return r;
}

// double -> float rounded to odd: a double rounding through this float and
// then to a format with at most 22 significand bits equals a single correct
// rounding of the double (the round-to-odd method).
__device__ __forceinline__ float f64_to_f32_odd(double d) {
    float f = (float)d;
    double back = (double)f;
    if (back != d && d == d) {
        uint32_t u = __float_as_uint(f);
        if (fabs(back) > fabs(d)) u -= 1u;   // rounded away from zero: step back
        u |= 1u;
        f = __uint_as_float(u);
    }
    return f;
}

// double -> float ahead of a rounding to FP16, by the bits of the double: the
// 29 significand bits that float drops are cleared and OR-ed into its lowest
// kept bit (round to odd), so that the conversion of the result is exact
// wherever float is normal.  Below that range FP16 rounds to zero either way,
// so the FP16 result equals that of f64_to_f32_odd.
__device__ __forceinline__ float f64_to_f32_odd_for_f16(double d) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(d);
    const uint32_t lo = (uint32_t)u;
    const uint32_t kept = (lo & 0xE0000000u) | (min(lo & 0x1FFFFFFFu, 1u) << 29);
    return (float)__longlong_as_double((long long)((u & 0xFFFFFFFF00000000ull) | kept));
}

// Workgroups are dealt round-robin to the 8 XCDs (workgroup b to XCD b mod 8).
// Renumber them so that each XCD takes a contiguous range of tiles and
// neighbouring tiles share that XCD's L2: the k-th workgroup of XCD j gets
// j q + min(j, r) + k, where nb = 8 q + r (a bijection of 0 .. nb-1).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, j = b & 7;
    return j * q + min(j, r) + (b >> 3);
}

// Round an accumulator value into storage format T (nearest even).
template <class T> struct Store;
template <> struct Store<double> {
    __device__ static double from_acc(double v) { return v; }
    __device__ static double from_f64(double v) { return v; }
};
template <> struct Store<float> {
    __device__ static float from_acc(float v) { return v; }
    __device__ static float from_f64(double v) { return (float)v; }
};
template <> struct Store<f16> {
    // The empty asm makes v opaque: without it the backend may fold the
    // producing FP32 FMA and this narrowing into one mixed-precision FMA that
    // rounds once instead of twice, so that the same source line would round
    // differently in different kernels.
    __device__ static f16 from_acc(float v) {
        asm volatile("" : "+v"(v));
        return (f16)v;
    }
    __device__ static f16 from_f64(double v) { return (f16)f64_to_f32_odd_for_f16(v); }
};
template <> struct Store<bf16> {
    __device__ static bf16 from_acc(float v) { return f32_to_bf16(v); }
    __device__ static bf16 from_f64(double v) { return f32_to_bf16(f64_to_f32_odd(v)); }
};

// Round a float or double into storage format T (a single correct rounding).
template <class T> __device__ __forceinline__ T store_as(double v) { return Store<T>::from_f64(v); }
template <class T> __device__ __forceinline__ T store_as(float v) { return Store<T>::from_acc((acc_t<T>)v); }

// Round a value of any accumulator type into T and widen it back: the value a
// store followed by a load would produce.
template <class T> __device__ __forceinline__ acc_t<T> round_to(float v) {
    return widen(Store<T>::from_acc((acc_t<T>)v));
}
template <class T> __device__ __forceinline__ acc_t<T> round_to(double v) {
    return widen(Store<T>::from_f64(v));
}

// Explicit fused multiply-add (the library is built with contraction off, so
// every other product and sum rounds separately and all kernels agree).
template <class A> __device__ __forceinline__ A fmaT(A a, A b, A c);
template <> __device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmaT<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// Row-vector loads and stores of V consecutive elements starting at an
// address aligned to V * sizeof(T) (guaranteed by the padded layout below).
template <int BYTES> struct RawChunk;
template <> struct RawChunk<2> { typedef uint16_t type; };
template <> struct RawChunk<4> { typedef uint32_t type; };
template <> struct RawChunk<8> { typedef uint2 type; };
template <> struct RawChunk<16> { typedef uint4 type; };

template <class T, int V, class A>
__device__ __forceinline__ void load_row(const T *__restrict__ p, A (&o)[V]) {
    constexpr int B = V * (int)sizeof(T);
    constexpr int CB = B >= 16 ? 16 : B;
    static_assert(B % CB == 0, "row bytes");
    typedef typename RawChunk<CB>::type C;
    union {
        C c[B / CB];
        T t[V];
    } u;
    const C *q = reinterpret_cast<const C *>(p);
#pragma unroll
    for (int i = 0; i < B / CB; ++i) u.c[i] = q[i];
#pragma unroll
    for (int i = 0; i < V; ++i) o[i] = (A)widen(u.t[i]);
}

template <class T, int V>
__device__ __forceinline__ void store_row(T *__restrict__ p, const T (&v)[V]) {
    constexpr int B = V * (int)sizeof(T);
    constexpr int CB = B >= 16 ? 16 : B;
    typedef typename RawChunk<CB>::type C;
    union {
        C c[B / CB];
        T t[V];
    } u;
#pragma unroll
    for (int i = 0; i < V; ++i) u.t[i] = v[i];
    C *q = reinterpret_cast<C *>(p);
#pragma unroll
    for (int i = 0; i < B / CB; ++i) q[i] = u.c[i];
}

// Raw (storage-format) row copies, for prefetching before conversion.
template <class T, int V> __device__ __forceinline__ void load_raw(const T *__restrict__ p, T (&v)[V]) {
    constexpr int B = V * (int)sizeof(T);
    constexpr int CB = B >= 16 ? 16 : B;
    typedef typename RawChunk<CB>::type C;
    union {
        C c[B / CB];
        T t[V];
    } u;
    const C *q = reinterpret_cast<const C *>(p);
#pragma unroll
    for (int i = 0; i < B / CB; ++i) u.c[i] = q[i];
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = u.t[i];
}

template <class T> __device__ __forceinline__ T zero_of() { return Store<T>::from_acc(acc_t<T>(0)); }

// ---------------------------------------------------------------------------
// Rows of values staged in LDS where thread t of a row holds the V values
// t V .. t V + V - 1.  Stored chunk-major: chunk j (C values, 16 bytes) of
// thread t sits at (j TXR + t) C, TXR the threads of a row, so the 16-byte
// accesses of a wave's lanes land on consecutive banks.  (Stored thread-major,
// lanes V sizeof(A) bytes apart, a 16-byte access of a wave touches each bank
// V sizeof(A) / 16 times.)  The arithmetic that uses the values is unchanged.
template <class A, int V> struct LdsRun {
    static constexpr int C = (16 / (int)sizeof(A)) < V ? 16 / (int)sizeof(A) : V;
    static constexpr int NC = V / C;
    static_assert(V % C == 0, "whole chunks per thread");
    // position of element x of the row
    __device__ __forceinline__ static int at(int x, int TXR) {
        const int t = x / V, i = x - t * V;
        return ((i / C) * TXR + t) * C + (i % C);
    }
    template <class S> __device__ __forceinline__ static void store(A *row, int t, int TXR, const S (&v)[V]) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            A c[C];
#pragma unroll
            for (int i = 0; i < C; ++i) {
                // (narrowing stores only values the format holds exactly)
                if constexpr (std::is_same<A, S>::value) c[i] = v[j * C + i];
                else c[i] = store_as<A>(v[j * C + i]);
            }
            store_row<A, C>(row + (size_t)(j * TXR + t) * C, c);
        }
    }
    template <class O> __device__ __forceinline__ static void load(const A *row, int t, int TXR, O (&v)[V]) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            O c[C];
            load_row<A, C>(row + (size_t)(j * TXR + t) * C, c);
#pragma unroll
            for (int i = 0; i < C; ++i) v[j * C + i] = c[i];
        }
    }
    // the last value of thread t - 1 and the first of thread t + 1
    __device__ __forceinline__ static A left_of(const A *row, int t, int TXR) {
        return row[((NC - 1) * TXR + t - 1) * C + C - 1];
    }
    __device__ __forceinline__ static A right_of(const A *row, int t, int TXR) { return row[(size_t)(t + 1) * C]; }
};

// A prefetched row kept packed in its storage format (e.g. eight FP16 values
// in four 32-bit registers) until it is widened.
template <class T, int V> struct RawRow {
    static constexpr int B = V * (int)sizeof(T);
    static constexpr int CB = B >= 16 ? 16 : B;
    typedef typename RawChunk<CB>::type C;
    C c[B / CB];
};

template <class T, int V> __device__ __forceinline__ void fetch_row(const T *__restrict__ p, RawRow<T, V> &r) {
    typedef typename RawRow<T, V>::C C;
    const C *q = reinterpret_cast<const C *>(p);
#pragma unroll
    for (int i = 0; i < RawRow<T, V>::B / RawRow<T, V>::CB; ++i) r.c[i] = q[i];
}

template <class T, int V> __device__ __forceinline__ void zero_row(RawRow<T, V> &r) {
    // all-zero bits are +0 in every storage format
    union {
        typename RawRow<T, V>::C c[RawRow<T, V>::B / RawRow<T, V>::CB];
        unsigned char bytes[RawRow<T, V>::B];
    } u;
#pragma unroll
    for (int i = 0; i < RawRow<T, V>::B; ++i) u.bytes[i] = 0;
#pragma unroll
    for (int i = 0; i < RawRow<T, V>::B / RawRow<T, V>::CB; ++i) r.c[i] = u.c[i];
}

template <class T, int V, class A> __device__ __forceinline__ void widen_row(const RawRow<T, V> &r, A (&o)[V]) {
    union {
        typename RawRow<T, V>::C c[RawRow<T, V>::B / RawRow<T, V>::CB];
        T t[V];
    } u;
#pragma unroll
    for (int i = 0; i < RawRow<T, V>::B / RawRow<T, V>::CB; ++i) u.c[i] = r.c[i];
#pragma unroll
    for (int i = 0; i < V; ++i) o[i] = (A)widen(u.t[i]);
}

// ---------------------------------------------------------------------------
// Padded level layout.  A level with n = 2^m - 1 interior points per
// dimension uses pitch P = 2^m.  Interior coordinates run 1..P-1; coordinate 0
// is a zero ghost.  Element (x, y, z) sits at (z*P + y)*P + x in 3-D and
// (z*P + x) in 2-D (the 2-D grid's rows are indexed by z).  Because the pitch
// is P, the ghost x = 0 of the next row doubles as the ghost x = P of this
// row, and row 0 of the next plane as row P of this plane; plane P is an
// explicit ghost plane, and one more plane of slack follows it.
template <int D> struct Grid {
    int P;
    __device__ __forceinline__ size_t at(int x, int y, int z) const {
        return D == 3 ? ((size_t)z * P + (size_t)y) * P + (size_t)x : (size_t)z * P + (size_t)x;
    }
    // true for rows that lie on the boundary or outside the interior
    __device__ __forceinline__ bool ghost_row(int y, int z) const {
        return z <= 0 || z >= P || (D == 3 && (y <= 0 || y >= P));
    }
};

// ---------------------------------------------------------------------------
// Q1 finite elements (bilinear in 2-D, trilinear in 3-D) in grid-scaled
// units: on every level the stiffness operator is the constant stencil S with
// 3 S = [8 centre, -1 on all 8 neighbours] (2-D) and 12 S = [32 centre, 0 on
// faces, -2 on the 12 edge neighbours, -1 on the 8 corners] (3-D).  q1_weighted
// returns 3 S v resp. 12 S v at padded offset o (integer weights, summed in A);
// multiply by q1_scale to get S v.  All neighbours of an interior point lie
// inside the padded array (ghosts hold zero).
template <int D, class A, class T>
__device__ __forceinline__ A q1_weighted(const T *__restrict__ v, size_t o, int P) {
    // one pointer per neighbour row; the x-neighbours are then constant offsets
    const T *c = v + o;
    const long Y = P;
    auto L = [](const T *r, int d) -> A { return (A)widen(r[d]); };
    if (D == 2) {
        const T *s = c - Y, *t = c + Y;
        const A nb = ((L(s, -1) + L(s, 0)) + (L(s, 1) + L(c, -1))) + ((L(c, 1) + L(t, -1)) + (L(t, 0) + L(t, 1)));
        return fmaT<A>(A(8), L(c, 0), -nb);
    }
    const long Z = (long)P * P;
    const T *bs = c - Z - Y, *b0 = c - Z, *bn = c - Z + Y, *s = c - Y, *t = c + Y;
    const T *ts = c + Z - Y, *t0 = c + Z, *tn = c + Z + Y;
    const A e = ((L(bs, 0) + L(b0, -1)) + (L(b0, 1) + L(bn, 0))) + ((L(s, -1) + L(s, 1)) + (L(t, -1) + L(t, 1))) +
                ((L(ts, 0) + L(t0, -1)) + (L(t0, 1) + L(tn, 0)));
    const A cn = ((L(bs, -1) + L(bs, 1)) + (L(bn, -1) + L(bn, 1))) + ((L(ts, -1) + L(ts, 1)) + (L(tn, -1) + L(tn, 1)));
    return fmaT<A>(A(32), L(c, 0), -fmaT<A>(A(2), e, cn));
}
template <int D, class A> __device__ __forceinline__ A q1_scale() { return D == 3 ? A(1.0 / 12.0) : A(1.0 / 3.0); }

// ---------------------------------------------------------------------------
// wave64 and block reductions with a fixed combination order.
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ void wave_reduce(double &s, double &m) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        m = nanmax(m, __shfl_xor(m, off, 64));
    }
}

// Reduce (sum, max) over the block; thread 0 gets the result.  Every thread
// of the block must call it.  Needs 2 * (blockDim.x / 64) doubles of LDS.
__device__ __forceinline__ void block_reduce(double &s, double &m, double *lds) {
    wave_reduce(s, m);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
        lds[2 * w] = s;
        lds[2 * w + 1] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ss = 0.0, mm = 0.0;
        for (int i = 0; i < nw; ++i) {
            ss += lds[2 * i];
            mm = nanmax(mm, lds[2 * i + 1]);
        }
        s = ss;
        m = mm;
    }
}

}  // namespace mg
