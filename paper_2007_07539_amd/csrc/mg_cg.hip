// Conjugate gradients on a base level of more than one point (the paper's
// base solver, Section 4.2): L x = b with the level's grid-scaled operator
// (the finite-difference stencil [2D, -1], or the Q1 stencil S), from x = 0, until ||r||_2 <= tol ||b||_2 or max_iter steps.  In
// grid-scaled units the residual of L x = b is the residual of the physical
// system, and CG is invariant under a scaling of the operator, so the steps
// are those of CG on the physical base system.  The base level is small and
// every step needs two reductions over all of it, so one workgroup does the
// whole solve; its vectors x, r, p, q live in the accumulator format (FP32 for
// FP32/FP16/BF16 levels, FP64 for FP64), dot products are summed in FP64 in a
// fixed order (deterministic), and x is rounded to the level format at the end.
#include "mg_device.h"
#include "mg_launch.h"

namespace mg {
namespace {

constexpr int kThreads = 1024;

// Sum over the workgroup, returned to every thread.
__device__ __forceinline__ double block_sum(double v, double *red, double *bc) {
    double m = 0.0;
    block_reduce(v, m, red);
    if (threadIdx.x == 0) bc[0] = v;
    __syncthreads();
    return bc[0];
}

template <int D, int OP, class T>
__global__ __launch_bounds__(kThreads) void k_cg_base(const T *__restrict__ b, T *__restrict__ c,
                                                      acc_t<T> *__restrict__ x, acc_t<T> *__restrict__ r,
                                                      acc_t<T> *__restrict__ p, acc_t<T> *__restrict__ q, int n, int P,
                                                      double tol, int max_iter) {
    typedef acc_t<T> A;
    __shared__ double red[2 * kThreads / 64];
    __shared__ double bc[1];
    const Grid<D> g{P};
    const long plane = D == 3 ? (long)P * P : (long)P;
    const long N = D == 3 ? (long)n * n * n : (long)n * n;
    auto pos = [&](long i) -> long {
        const int xx = (int)(i % n) + 1;
        const long rest = i / n;
        if (D == 3) return (long)g.at(xx, (int)(rest % n) + 1, (int)(rest / n) + 1);
        return (long)g.at(xx, 0, (int)rest + 1);
    };
    double loc = 0.0;
    for (long i = threadIdx.x; i < N; i += kThreads) {
        const long o = pos(i);
        const A bi = (A)widen(b[o]);
        x[o] = A(0);
        r[o] = bi;
        p[o] = bi;
        loc += (double)bi * (double)bi;
    }
    double rr = block_sum(loc, red, bc);
    const double stop = tol * sqrt(rr);
    for (int k = 0; k < max_iter && sqrt(rr) > stop; ++k) {
        __syncthreads();  // every p of the last step is written
        loc = 0.0;
        for (long i = threadIdx.x; i < N; i += kThreads) {
            const long o = pos(i);
            A lp;
            if (OP == 1) {
                lp = q1_weighted<D, A>(p, (size_t)o, P) * q1_scale<D, A>();
            } else {
                A nb = p[o - 1] + p[o + 1];
                if (D == 3) {
                    nb += p[o - P];
                    nb += p[o + P];
                }
                nb += p[o - plane];
                nb += p[o + plane];
                lp = fmaT<A>(A(2 * D), p[o], -nb);
            }
            q[o] = lp;
            loc += (double)p[o] * (double)lp;
        }
        const double pq = block_sum(loc, red, bc);
        if (!(pq > 0.0)) break;  // p = 0: the residual is already zero
        const A a = (A)(rr / pq);
        loc = 0.0;
        for (long i = threadIdx.x; i < N; i += kThreads) {
            const long o = pos(i);
            x[o] = fmaT<A>(a, p[o], x[o]);
            const A ri = fmaT<A>(-a, q[o], r[o]);
            r[o] = ri;
            loc += (double)ri * (double)ri;
        }
        const double rr_new = block_sum(loc, red, bc);
        const A beta = (A)(rr_new / rr);
        __syncthreads();  // every q of this step has been read
        for (long i = threadIdx.x; i < N; i += kThreads) {
            const long o = pos(i);
            p[o] = fmaT<A>(beta, p[o], r[o]);
        }
        rr = rr_new;
    }
    for (long i = threadIdx.x; i < N; i += kThreads) {
        const long o = pos(i);
        c[o] = Store<T>::from_acc(x[o]);
    }
}

template <int OP, class T>
hipError_t cg_t(int D, int n, int P, const void *b, void *c, void *scratch, size_t stride, double tol, int max_iter,
                hipStream_t st) {
    typedef acc_t<T> A;
    A *x = static_cast<A *>(scratch);
    A *r = reinterpret_cast<A *>(static_cast<char *>(scratch) + stride);
    A *p = reinterpret_cast<A *>(static_cast<char *>(scratch) + 2 * stride);
    A *q = reinterpret_cast<A *>(static_cast<char *>(scratch) + 3 * stride);
    if (D == 3)
        hipLaunchKernelGGL((k_cg_base<3, OP, T>), dim3(1), dim3(kThreads), 0, st, static_cast<const T *>(b),
                           static_cast<T *>(c), x, r, p, q, n, P, tol, max_iter);
    else
        hipLaunchKernelGGL((k_cg_base<2, OP, T>), dim3(1), dim3(kThreads), 0, st, static_cast<const T *>(b),
                           static_cast<T *>(c), x, r, p, q, n, P, tol, max_iter);
    return hipGetLastError();
}

}  // namespace

size_t cg_scratch_stride(int prec, size_t elems) {
    const size_t acc = prec == P_F64 ? sizeof(double) : sizeof(float);
    return (elems * acc + 255) / 256 * 256;
}

template <int OP>
hipError_t cg_op(int D, int prec, int n, int P, const void *b, void *c, void *scratch, size_t stride, double tol,
                 int max_iter, hipStream_t st) {
    switch (prec) {
    case P_F64: return cg_t<OP, double>(D, n, P, b, c, scratch, stride, tol, max_iter, st);
    case P_F32: return cg_t<OP, float>(D, n, P, b, c, scratch, stride, tol, max_iter, st);
    case P_F16: return cg_t<OP, f16>(D, n, P, b, c, scratch, stride, tol, max_iter, st);
    case P_BF16: return cg_t<OP, bf16>(D, n, P, b, c, scratch, stride, tol, max_iter, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_cg_base(int D, int prec, int n, int P, const void *b, void *c, void *scratch, size_t stride,
                          double tol, int max_iter, int op, hipStream_t st) {
    if (n < 2 || (D != 2 && D != 3)) return hipErrorInvalidValue;
    return op == 1 ? cg_op<1>(D, prec, n, P, b, c, scratch, stride, tol, max_iter, st)
                   : cg_op<0>(D, prec, n, P, b, c, scratch, stride, tol, max_iter, st);
}

}  // namespace mg
