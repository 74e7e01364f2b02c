// Residual rescaling on restriction into a half-precision level (Section 6:
// the DSH_MG variant rescales the residual when it restricts into its FP16
// levels, as Algorithm 2 scales the finest level's residual before the cast).
// With t the restricted residual, kept in the fine level's accumulator format:
//   way down:  s = max |t|,  b_c = round_T(t * (1/s))
//   way up:    e = s * c_c, in the fine accumulator format, then the usual
//              prolongation + correction + sweep reads e instead of c_c.
// In exact arithmetic the V-cycle is linear in its right-hand side, so the
// result is unchanged; in half precision the coarse residual keeps its
// significant digits instead of drifting into the subnormal range.
#include "mg_device.h"
#include "mg_launch.h"

namespace mg {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxParts = 1024;

template <class TA>
__global__ __launch_bounds__(kThreads) void k_absmax_part(const TA *__restrict__ t, long n, double *__restrict__ part) {
    __shared__ double red[2 * kThreads / 64];
    double s = 0.0, m = 0.0;
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads)
        m = nanmax(m, fabs((double)t[i]));
    block_reduce(s, m, red);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// s and 1/s of the level (a zero or non-finite maximum leaves s = 1, as the
// finest level's scaling does).
__global__ __launch_bounds__(kThreads) void k_absmax_fin(const double *__restrict__ part, int nparts,
                                                         double *__restrict__ rs) {
    __shared__ double red[2 * kThreads / 64];
    double s = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) m = nanmax(m, part[i]);
    block_reduce(s, m, red);
    if (threadIdx.x == 0) {
        double a = m;
        if (!(a > 0.0) || a > 1.7e308) a = 1.0;
        rs[0] = a;
        rs[1] = 1.0 / a;
    }
}

template <class TA, class T>
__global__ __launch_bounds__(kThreads) void k_scale_cast(const TA *__restrict__ t, const double *__restrict__ rs,
                                                         T *__restrict__ out, long n) {
    const double inv = rs[1];
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads)
        out[i] = Store<T>::from_f64((double)t[i] * inv);
}

template <class T, class TA>
__global__ __launch_bounds__(kThreads) void k_scale_widen(const T *__restrict__ c, const double *__restrict__ rs,
                                                          TA *__restrict__ out, long n) {
    const double s = rs[0];
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads)
        out[i] = Store<TA>::from_f64(s * (double)widen(c[i]));
}

int grid_for(long n) { return (int)std::max<long>(1, std::min<long>(kMaxParts, (n + kThreads - 1) / kThreads)); }

template <class TA>
hipError_t absmax_t(const void *t, long n, double *part, double *rs, hipStream_t st) {
    const int blocks = grid_for(n);
    hipLaunchKernelGGL((k_absmax_part<TA>), dim3(blocks), dim3(kThreads), 0, st, static_cast<const TA *>(t), n,
                       part);
    hipLaunchKernelGGL(k_absmax_fin, dim3(1), dim3(kThreads), 0, st, part, blocks, rs);
    return hipGetLastError();
}

template <class TA, class T>
hipError_t scale_cast_t(const void *t, const double *rs, void *out, long n, hipStream_t st) {
    hipLaunchKernelGGL((k_scale_cast<TA, T>), dim3(grid_for(n)), dim3(kThreads), 0, st, static_cast<const TA *>(t),
                       rs, static_cast<T *>(out), n);
    return hipGetLastError();
}

template <class T, class TA>
hipError_t scale_widen_t(const void *c, const double *rs, void *out, long n, hipStream_t st) {
    hipLaunchKernelGGL((k_scale_widen<T, TA>), dim3(grid_for(n)), dim3(kThreads), 0, st, static_cast<const T *>(c),
                       rs, static_cast<TA *>(out), n);
    return hipGetLastError();
}

}  // namespace

size_t rescale_part_count() { return kMaxParts; }

hipError_t launch_absmax(int pa, const void *t, long n, double *part, double *rs, hipStream_t st) {
    switch (pa) {
    case P_F64: return absmax_t<double>(t, n, part, rs, st);
    case P_F32: return absmax_t<float>(t, n, part, rs, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scale_cast(int pa, int prec, const void *t, const double *rs, void *out, long n, hipStream_t st) {
    if (pa == P_F64) {
        switch (prec) {
        case P_F16: return scale_cast_t<double, f16>(t, rs, out, n, st);
        case P_BF16: return scale_cast_t<double, bf16>(t, rs, out, n, st);
        }
    } else if (pa == P_F32) {
        switch (prec) {
        case P_F16: return scale_cast_t<float, f16>(t, rs, out, n, st);
        case P_BF16: return scale_cast_t<float, bf16>(t, rs, out, n, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scale_widen(int prec, int pa, const void *c, const double *rs, void *out, long n, hipStream_t st) {
    if (pa == P_F64) {
        switch (prec) {
        case P_F16: return scale_widen_t<f16, double>(c, rs, out, n, st);
        case P_BF16: return scale_widen_t<bf16, double>(c, rs, out, n, st);
        }
    } else if (pa == P_F32) {
        switch (prec) {
        case P_F16: return scale_widen_t<f16, float>(c, rs, out, n, st);
        case P_BF16: return scale_widen_t<bf16, float>(c, rs, out, n, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace mg
