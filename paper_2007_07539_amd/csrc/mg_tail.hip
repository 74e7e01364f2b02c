// The coarse end of the 3-D V-cycle in one workgroup: every level from a
// small grid (pitch 16 or 8) down to the one-point base level and back up,
// with all level vectors held in LDS.  On the coarse levels each stage is
// a few thousand points, so as separate launches they cost launch latency,
// not bandwidth; here a stage costs one pass over LDS and a barrier.
//
// The arithmetic is the level kernels' own, operation for operation: the
// neighbour sum order (x-, x+, y-, y+, z-, z+), the explicit FMAs of the
// Jacobi sweep, the residual and full-weighting order of the restriction,
// the canonical interpolation sum order of the prolongation, and rounding to
// each level's storage format wherever a level kernel stores a value.  So a
// V-cycle with the fused tail is bitwise the one without it.
#include "mg_device.h"
#include "mg_launch.h"

#include <type_traits>

namespace mg {
namespace {

// LDS copy of a level: (P + 1) planes of P x P (interior 1..P-1, zero
// ghosts, plane P zero); x = P and y = P alias the next row and plane.
__device__ __forceinline__ int lid(int P, int x, int y, int z) { return (z * P + y) * P + x; }

template <class T> __device__ __forceinline__ acc_t<T> at(const T *a, int P, int x, int y, int z) {
    return (acc_t<T>)widen(a[lid(P, x, y, z)]);
}

struct Pt {
    int x, y, z;
};
// Item i of a P^3 sweep (P = 2^lg): x fastest; ghost positions (a zero
// coordinate) are skipped by the caller.
__device__ __forceinline__ Pt point(int i, int lg) {
    const int m = (1 << lg) - 1;
    return Pt{i & m, (i >> lg) & m, i >> (2 * lg)};
}
__device__ __forceinline__ bool ghost(const Pt &p) { return p.x == 0 || p.y == 0 || p.z == 0; }
__device__ __forceinline__ int lg2(int P) { return 31 - __clz(P); }

// c1 = round_T(k b): the first Jacobi iterate from zero.
template <class T> __device__ void st_jac0(const T *b, T *c, int P, acc_t<T> k) {
    const int lg = lg2(P), N = P * P * P;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const Pt p = point(i, lg);
        if (ghost(p)) continue;
        c[lid(P, p.x, p.y, p.z)] = Store<T>::from_acc(k * at(b, P, p.x, p.y, p.z));
    }
}

template <class T> __device__ __forceinline__ acc_t<T> nbsum(const T *c, int P, int x, int y, int z) {
    acc_t<T> nb = at(c, P, x - 1, y, z) + at(c, P, x + 1, y, z);
    nb += at(c, P, x, y - 1, z);
    nb += at(c, P, x, y + 1, z);
    nb += at(c, P, x, y, z - 1);
    nb += at(c, P, x, y, z + 1);
    return nb;
}

// co = round_T(c + k (b - (6 c - nb))).
template <class T> __device__ void st_sweep(const T *b, const T *c, T *co, int P, acc_t<T> k) {
    typedef acc_t<T> A;
    const int lg = lg2(P), N = P * P * P;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const Pt p = point(i, lg);
        if (ghost(p)) continue;
        const A cc = at(c, P, p.x, p.y, p.z);
        const A lc = fmaT<A>(A(6), cc, -nbsum(c, P, p.x, p.y, p.z));
        co[lid(P, p.x, p.y, p.z)] = Store<T>::from_acc(fmaT<A>(k, at(b, P, p.x, p.y, p.z) - lc, cc));
    }
}

// bc = round_TC(FW(b - L c)), fine residuals in the fine accumulator, in the
// order of the level kernels: x weights per fine row, then y, then z.  Two
// passes: rx(X, y, z) = x-weighted residuals into the scratch array (the free
// correction buffer of the level), then the y and z weights per coarse point.
template <class TF>
__device__ __forceinline__ acc_t<TF> resid(const TF *b, const TF *c, int P, int x, int y, int z) {
    typedef acc_t<TF> A;
    return at(b, P, x, y, z) - fmaT<A>(A(6), at(c, P, x, y, z), -nbsum(c, P, x, y, z));
}

template <class TF, class TC>
__device__ void st_restrict(const TF *b, const TF *c, TC *bc, acc_t<TF> *rx, int P) {
    typedef acc_t<TF> A;
    const int lg = lg2(P), Pc = P / 2;
    for (int i = threadIdx.x; i < Pc * P * P; i += blockDim.x) {
        const int X = i & (Pc - 1), y = (i >> (lg - 1)) & (P - 1), z = i >> (2 * lg - 1);
        if (X == 0 || y == 0 || z == 0) continue;
        const A r0 = resid(b, c, P, 2 * X - 1, y, z), r1 = resid(b, c, P, 2 * X, y, z),
                r2 = resid(b, c, P, 2 * X + 1, y, z);
        rx[(z * P + y) * Pc + X] = A(0.25) * (r0 + r2) + A(0.5) * r1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Pc * Pc * Pc; i += blockDim.x) {
        const Pt q = point(i, lg - 1);
        if (ghost(q)) continue;
        A acc = A(0), v = A(0);
        for (int j = 0; j < 3; ++j) {
            const int zf = 2 * q.z - 1 + j;
            const A *row = rx + (zf * P + 2 * q.y - 1) * Pc + q.x;
            const A qq = A(0.25) * (row[0] + row[2 * Pc]) + A(0.5) * row[Pc];
            if (j == 0) {
                acc = A(0.25) * qq;
            } else if (j == 1) {
                acc += A(0.5) * qq;
            } else {
                v = acc + A(0.25) * qq;
            }
        }
        bc[lid(Pc, q.x, q.y, q.z)] = store_as<TC>(v);
    }
}

// f = round_TF(c + 4 P e): linear interpolation in the canonical order (per
// contributing coarse row the z sum over interior coarse planes, then the y
// weights, then the x weights), in FP64 when either level is FP64.
template <class TF, class TC> struct Interp {
    typedef typename std::conditional<std::is_same<TC, double>::value || std::is_same<TF, double>::value, double,
                                      float>::type PA;
    __device__ static int split(int q, int (&Q)[2]) {
        if ((q & 1) == 0) {
            Q[0] = q >> 1;
            return 1;
        }
        Q[0] = (q - 1) >> 1;
        Q[1] = (q + 1) >> 1;
        return 2;
    }
    __device__ static PA colsum(const TC *ec, int Pc, int X, int y, int z) {
        PA s = PA(0);
        int Zs[2], Ys[2];
        const int nz = split(z, Zs), ny = split(y, Ys);
        const PA wz = nz == 1 ? PA(1) : PA(0.5), wy = ny == 1 ? PA(1) : PA(0.5);
        for (int bb = 0; bb < ny; ++bb) {
            const int Y = Ys[bb];
            PA t = PA(0);
            if (X >= 1 && X < Pc && Y >= 1 && Y < Pc) {
                for (int a = 0; a < nz; ++a) {
                    const int Z = Zs[a];
                    if (Z < 1 || Z >= Pc) continue;
                    t += wz * (PA)widen(ec[lid(Pc, X, Y, Z)]);
                }
            }
            s += wy * t;
        }
        return s;
    }
};

template <class TF, class TC> __device__ void st_prolong(const TF *c, const TC *ec, TF *f, int P) {
    typedef Interp<TF, TC> I;
    typedef typename I::PA PA;
    // every position, ghosts included: f's buffer held the restriction's
    // scratch values, and its ghosts must read as zero again
    const int lg = lg2(P), N = (P + 1) * P * P, Pc = P / 2;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const Pt p = point(i, lg);
        if (ghost(p) || p.z == P) {
            f[i] = Store<TF>::from_acc(acc_t<TF>(0));
            continue;
        }
        PA e;
        if ((p.x & 1) == 0) {
            e = I::colsum(ec, Pc, p.x >> 1, p.y, p.z);
        } else {
            e = PA(0.5) * (I::colsum(ec, Pc, (p.x - 1) >> 1, p.y, p.z) + I::colsum(ec, Pc, (p.x + 1) >> 1, p.y, p.z));
        }
        const PA v = (PA)at(c, P, p.x, p.y, p.z) + PA(4) * e;
        f[lid(P, p.x, p.y, p.z)] = store_as<TF>(v);
    }
}

__device__ __forceinline__ int lds_elems(int P) { return (P + 1) * P * P; }

template <class T> __device__ void zero_lds(T *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = Store<T>::from_acc(acc_t<T>(0));
}

// Levels: nlev grids of type T with pitches P0, P0/2, ..., 4, then the base
// (pitch 2) of type TB.  Reads the right-hand side of the first from b_in
// (padded HBM layout, pitch P0) and writes its corrected correction to c_out.
template <class T, class TB>
__global__ __launch_bounds__(1024) void k_tail(const T *__restrict__ b_in, T *__restrict__ c_out, int P0, int nlev,
                                                int nu1, int nu2, double omega) {
    extern __shared__ __align__(16) unsigned char smem[];
    typedef acc_t<T> A;
    const A k = (A)(omega / 6.0);
    // carve: per level b, c0, c1 (T), then the base b, c (TB); addresses are
    // recomputed from the level index (no per-thread pointer tables)
    auto level_off = [&](int l) {
        size_t off = 0;
        for (int i = 0; i < l; ++i) off = (off + 3 * (size_t)lds_elems(P0 >> i) * sizeof(T) + 15) & ~(size_t)15;
        return off;
    };
    auto arr = [&](int l, int j) {
        return reinterpret_cast<T *>(smem + level_off(l) + (size_t)j * lds_elems(P0 >> l) * sizeof(T));
    };
    TB *bb = reinterpret_cast<TB *>(smem + level_off(nlev));
    TB *bcv = bb + lds_elems(2);
    for (int l = 0; l < nlev; ++l) zero_lds(arr(l, 0), 3 * lds_elems(P0 >> l));
    zero_lds(bb, 2 * lds_elems(2));
    __syncthreads();
    {
        const int n0 = lds_elems(P0);
        T *b0 = arr(0, 0);
        for (int i = threadIdx.x; i < n0; i += blockDim.x) b0[i] = b_in[i];
    }
    __syncthreads();
    unsigned curbits = 0;  // bit l set: level l's current correction is array 2, else array 1
    // down: pre-smoothing and restriction
    for (int l = 0; l < nlev; ++l) {
        const int P = P0 >> l;
        T *b = arr(l, 0);
        st_jac0(b, arr(l, 2), P, k);
        __syncthreads();
        int c = 2;
        if (nu1 >= 2) {
            st_sweep(b, arr(l, 2), arr(l, 1), P, k);
            __syncthreads();
            c = 1;
            for (int s = 2; s < nu1; ++s) {
                st_sweep(b, arr(l, c), arr(l, 3 - c), P, k);
                __syncthreads();
                c = 3 - c;
            }
        }
        if (c == 2) curbits |= 1u << l;
        A *rx = reinterpret_cast<A *>(arr(l, 3 - c));  // free during the restriction
        if (l + 1 < nlev) {
            st_restrict<T, T>(b, arr(l, c), arr(l + 1, 0), rx, P);
        } else {
            st_restrict<T, TB>(b, arr(l, c), bb, rx, P);
        }
        __syncthreads();
    }
    // base: c = b / 6 at the single interior point
    if (threadIdx.x == 0) {
        typedef acc_t<TB> AB;
        bcv[lid(2, 1, 1, 1)] = Store<TB>::from_acc(widen(bb[lid(2, 1, 1, 1)]) / AB(6));
    }
    __syncthreads();
    // up: prolongation, correction and post-smoothing
    for (int l = nlev - 1; l >= 0; --l) {
        const int P = P0 >> l;
        T *b = arr(l, 0);
        int c = (curbits >> l) & 1u ? 2 : 1;
        if (l + 1 < nlev) {
            const int cc = (curbits >> (l + 1)) & 1u ? 2 : 1;
            st_prolong<T, T>(arr(l, c), arr(l + 1, cc), arr(l, 3 - c), P);
        } else {
            st_prolong<T, TB>(arr(l, c), bcv, arr(l, 3 - c), P);
        }
        __syncthreads();
        c = 3 - c;  // the corrected correction
        for (int s = 0; s < nu2; ++s) {
            st_sweep(b, arr(l, c), arr(l, 3 - c), P, k);
            __syncthreads();
            c = 3 - c;
        }
        curbits = (curbits & ~(1u << l)) | (c == 2 ? 1u << l : 0u);
    }
    {
        const int n0 = lds_elems(P0);
        const T *src = arr(0, (curbits & 1u) ? 2 : 1);
        for (int i = threadIdx.x; i < n0; i += blockDim.x) c_out[i] = src[i];
    }
}

template <class T, class TB> size_t tail_bytes(int P0, int nlev) {
    size_t off = 0;
    for (int l = 0; l < nlev; ++l) {
        const int P = P0 >> l;
        off += 3 * (size_t)(P + 1) * P * P * sizeof(T);
        off = (off + 15) & ~(size_t)15;
    }
    return off + 2 * (size_t)(3 * 2 * 2) * sizeof(TB);
}

#define MG_TT(prec, ...)                                   \
    switch (prec) {                                        \
    case P_F64: { typedef double TX; __VA_ARGS__; break; } \
    case P_F32: { typedef float TX; __VA_ARGS__; break; }  \
    case P_F16: { typedef f16 TX; __VA_ARGS__; break; }    \
    case P_BF16: { typedef bf16 TX; __VA_ARGS__; break; }  \
    default: break;                                        \
    }

template <class T>
hipError_t tail_t(int pb, int P0, int nlev, const void *b, void *c, int nu1, int nu2, double omega, hipStream_t st,
                  size_t *bytes_only) {
    MG_TT(pb, {
        const size_t lds = tail_bytes<T, TX>(P0, nlev);
        if (bytes_only) {
            *bytes_only = lds;
            return hipSuccess;
        }
        hipLaunchKernelGGL((k_tail<T, TX>), dim3(1), dim3(1024), lds, st, static_cast<const T *>(b),
                           static_cast<T *>(c), P0, nlev, nu1, nu2, omega);
        return hipGetLastError();
    });
    return hipErrorInvalidValue;
}

hipError_t tail_dispatch(int prec, int pb, int P0, int nlev, const void *b, void *c, int nu1, int nu2, double omega,
                         hipStream_t st, size_t *bytes_only) {
    if (nlev < 1 || nlev > 6 || P0 != (4 << (nlev - 1))) return hipErrorInvalidValue;
    switch (prec) {
    case P_F64: return tail_t<double>(pb, P0, nlev, b, c, nu1, nu2, omega, st, bytes_only);
    case P_F32: return tail_t<float>(pb, P0, nlev, b, c, nu1, nu2, omega, st, bytes_only);
    case P_F16: return tail_t<f16>(pb, P0, nlev, b, c, nu1, nu2, omega, st, bytes_only);
    case P_BF16: return tail_t<bf16>(pb, P0, nlev, b, c, nu1, nu2, omega, st, bytes_only);
    }
    return hipErrorInvalidValue;
}

}  // namespace

size_t tail_lds_bytes(int prec, int pb, int P0, int nlev) {
    size_t bytes = 0;
    if (tail_dispatch(prec, pb, P0, nlev, nullptr, nullptr, 0, 0, 0.0, nullptr, &bytes) != hipSuccess) return 0;
    return bytes;
}

hipError_t launch_tail(int prec, int pb, int P0, int nlev, const void *b, void *c, int nu1, int nu2, double omega,
                       hipStream_t st) {
    const size_t lds = tail_lds_bytes(prec, pb, P0, nlev);
    if (lds == 0 || lds > 65536 || nu1 < 1 || nu2 < 1) return hipErrorInvalidValue;
    return tail_dispatch(prec, pb, P0, nlev, b, c, nu1, nu2, omega, st, nullptr);
}

}  // namespace mg
