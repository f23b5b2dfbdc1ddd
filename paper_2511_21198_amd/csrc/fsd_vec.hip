// Vector, reduction and single-workgroup scalar kernels of the Krylov loops.
//
// Reductions are two-stage and deterministic: every workgroup writes one
// float64 partial sum (wavefront shuffles, then LDS across waves) and a
// single-workgroup scalar kernel adds the partials in a fixed order, so a
// repeated run gives bitwise identical iterates.  All dot products and norms
// accumulate in float64 whatever the vector type.
#include "fsd_vec.h"

namespace fsd {

namespace {

constexpr int VT = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline double block_sum_vt(double v, double* sbuf) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sbuf[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < VT / 64; ++i) s += sbuf[i];
    }
    return s;
}

__device__ inline bool is_finite(double v) { return __builtin_isfinite(v); }

template <typename T>
__global__ __launch_bounds__(VT) void k_pack(const double* __restrict__ dense, T* __restrict__ pad,
                                             int n1, int P1, long rows, double scale) {
    const long total = rows * P1;
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < total; e += (long)gridDim.x * VT) {
        const long row = e / P1;
        const int x = (int)(e - row * P1);
        pad[e] = x < n1 ? (T)(scale * dense[row * n1 + x]) : T(0);
    }
}

template <typename T>
__global__ __launch_bounds__(VT) void k_unpack(const T* __restrict__ pad, double* __restrict__ dense,
                                               int n1, int P1, long rows) {
    const long total = rows * n1;
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < total; e += (long)gridDim.x * VT) {
        const long row = e / n1;
        const int x = (int)(e - row * n1);
        dense[e] = (double)pad[row * P1 + x];
    }
}

template <typename T>
__global__ __launch_bounds__(VT) void k_dot(const T* __restrict__ a, const T* __restrict__ b, long N,
                                            double* __restrict__ partials, const Ctrl* ctrl) {
    __shared__ double sb[VT / 64];
    if (ctrl && ctrl->done) return;
    double acc = 0.0;
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT)
        acc += (double)a[e] * (double)b[e];
    const double s = block_sum_vt(acc, sb);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// x += alpha p ; r -= alpha q ; partial ||r||^2   (alpha from ctrl)
template <typename T>
__global__ __launch_bounds__(VT) void k_update_xr(T* __restrict__ x, T* __restrict__ r,
                                                  const T* __restrict__ p, const T* __restrict__ q,
                                                  long N, const Ctrl* ctrl,
                                                  double* __restrict__ partials) {
    __shared__ double sb[VT / 64];
    if (ctrl->done) return;
    const T alpha = (T)ctrl->alpha;
    double acc = 0.0;
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT) {
        x[e] += alpha * p[e];
        const T rv = r[e] - alpha * q[e];
        r[e] = rv;
        acc += (double)rv * (double)rv;
    }
    const double s = block_sum_vt(acc, sb);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(VT) void k_cast(const Tin* __restrict__ in, Tout* __restrict__ out, long N,
                                             double scale) {
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT)
        out[e] = (Tout)(scale * (double)in[e]);
}

// x += scale * d (x float64, d any type)
template <typename Td>
__global__ __launch_bounds__(VT) void k_axpy64(double* __restrict__ x, const Td* __restrict__ d, long N,
                                               double scale) {
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT)
        x[e] += scale * (double)d[e];
}

// x += d (same type)
template <typename T>
__global__ __launch_bounds__(VT) void k_add(T* __restrict__ x, const T* __restrict__ d, long N) {
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT) x[e] += d[e];
}

template <typename T>
__global__ __launch_bounds__(VT) void k_fill(T* __restrict__ x, long N, T v) {
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT) x[e] = v;
}

template <typename T>
__global__ __launch_bounds__(VT) void k_copy(const T* __restrict__ a, T* __restrict__ b, long N) {
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT) b[e] = a[e];
}

__global__ __launch_bounds__(VT) void k_extrap(double* __restrict__ x, double* __restrict__ up, long N,
                                               int have) {
    for (long e = blockIdx.x * (long)VT + threadIdx.x; e < N; e += (long)gridDim.x * VT) {
        const double un = x[e];
        if (have) x[e] = 2.0 * un - up[e];
        up[e] = un;
    }
}

__global__ void k_ctrl_init(Ctrl* c, double tol2, int maxit, int restart, double abs2,
                            double eta2) {
    if (threadIdx.x == 0) {
        c->bb = 0; c->rr = 0; c->rz = 0; c->pq = 0; c->alpha = 0; c->beta = 0;
        c->thresh = 0; c->tol2 = tol2; c->iters = 0; c->maxit = maxit; c->done = 0;
        c->status = 0; c->first = 1; c->gm_j = 0; c->gm_m = restart; c->gm_k = 0;
        c->gm_beta = 0; c->gm_hnext = 0; c->gm_scale = 0; c->abs2 = abs2;
        c->gm_w2 = 0; c->gm_wp2 = 0; c->gm_eta2 = eta2; c->gm_reorth = 0; c->gm_nreorth = 0;
        for (int j = 0; j < kMaxRestart; ++j) c->gm_rflag[j] = 0;
    }
}

// Single-workgroup scalar step: S = sum of the partials in a fixed order,
// then the Krylov scalar update selected by op.
__global__ __launch_bounds__(VT) void k_scalar(Ctrl* c, const double* __restrict__ partials, int nparts,
                                               int op) {
    __shared__ double sb[VT / 64];
    if (c->done) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += VT) acc += partials[i];
    const double S = block_sum_vt(acc, sb);
    if (threadIdx.x != 0) return;
    switch (op) {
        case SC_BB:
            c->bb = S;
            c->thresh = fmax(c->tol2 * S, c->abs2);
            if (!is_finite(S)) { c->status = 4; c->done = 1; }
            else if (S == 0.0) { c->rr = 0.0; c->done = 1; }
            break;
        case SC_RR0:
            c->rr = S;
            if (!is_finite(S)) { c->status = 4; c->done = 1; }
            else if (S <= c->thresh) c->done = 1;
            break;
        case SC_RZ0:
            c->rz = S;
            c->first = 1;
            if (!is_finite(S)) { c->status = 4; c->done = 1; }
            break;
        case SC_ALPHA:
            c->pq = S;
            if (!is_finite(S)) { c->status = 4; c->done = 1; }
            else if (!(S > 0.0)) { c->status = 3; c->done = 1; }
            else c->alpha = c->rz / S;
            break;
        case SC_CHECK:
            c->rr = S;
            c->iters += 1;
            if (!is_finite(S)) { c->status = 4; c->done = 1; }
            else if (S <= c->thresh) c->done = 1;
            else if (c->iters >= c->maxit) { c->status = 2; c->done = 1; }
            break;
        case SC_BETA:
            if (!is_finite(S)) { c->status = 4; c->done = 1; break; }
            c->beta = S / c->rz;
            c->rz = S;
            c->first = 0;
            break;
        case SC_STORE:
            c->pq = S;
            break;
        default:
            break;
    }
}

inline int vgrid(long N) {
    long g = (N + VT * 4 - 1) / (VT * 4);
    if (g > kVecGrid) g = kVecGrid;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int vec_grid(long N) { return vgrid(N); }

template <typename T>
hipError_t vec_pack(const double* dense, T* pad, int n1, int P1, long rows, double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_pack<T>), dim3(vgrid(rows * P1)), dim3(VT), 0, s, dense, pad, n1, P1, rows, scale);
    return hipGetLastError();
}
template <typename T>
hipError_t vec_unpack(const T* pad, double* dense, int n1, int P1, long rows, hipStream_t s) {
    hipLaunchKernelGGL((k_unpack<T>), dim3(vgrid(rows * n1)), dim3(VT), 0, s, pad, dense, n1, P1, rows);
    return hipGetLastError();
}
template <typename T>
hipError_t vec_dot(const T* a, const T* b, long N, double* partials, const Ctrl* ctrl, int* nparts,
                   hipStream_t s) {
    const int g = vgrid(N);
    *nparts = g;
    hipLaunchKernelGGL((k_dot<T>), dim3(g), dim3(VT), 0, s, a, b, N, partials, ctrl);
    return hipGetLastError();
}
template <typename T>
hipError_t vec_update_xr(T* x, T* r, const T* p, const T* q, long N, const Ctrl* ctrl,
                         double* partials, int* nparts, hipStream_t s) {
    const int g = vgrid(N);
    *nparts = g;
    hipLaunchKernelGGL((k_update_xr<T>), dim3(g), dim3(VT), 0, s, x, r, p, q, N, ctrl, partials);
    return hipGetLastError();
}
template <typename Tin, typename Tout>
hipError_t vec_cast(const Tin* in, Tout* out, long N, double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3(vgrid(N)), dim3(VT), 0, s, in, out, N, scale);
    return hipGetLastError();
}
template <typename Td>
hipError_t vec_axpy64(double* x, const Td* d, long N, double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_axpy64<Td>), dim3(vgrid(N)), dim3(VT), 0, s, x, d, N, scale);
    return hipGetLastError();
}
template <typename T>
hipError_t vec_axpy(T* x, const T* d, long N, hipStream_t s) {
    hipLaunchKernelGGL((k_add<T>), dim3(vgrid(N)), dim3(VT), 0, s, x, d, N);
    return hipGetLastError();
}
template <typename T>
hipError_t vec_fill(T* x, long N, T v, hipStream_t s) {
    hipLaunchKernelGGL((k_fill<T>), dim3(vgrid(N)), dim3(VT), 0, s, x, N, v);
    return hipGetLastError();
}
template <typename T>
hipError_t vec_copy(const T* a, T* b, long N, hipStream_t s) {
    hipLaunchKernelGGL((k_copy<T>), dim3(vgrid(N)), dim3(VT), 0, s, a, b, N);
    return hipGetLastError();
}
hipError_t vec_extrap(double* x, double* up, long N, int have, hipStream_t s) {
    hipLaunchKernelGGL(k_extrap, dim3(vgrid(N)), dim3(VT), 0, s, x, up, N, have);
    return hipGetLastError();
}
hipError_t ctrl_init(Ctrl* c, double tol2, int maxit, int restart, hipStream_t s, double abs2,
                     double eta2) {
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, s, c, tol2, maxit, restart, abs2, eta2);
    return hipGetLastError();
}
hipError_t scalar_step(Ctrl* c, const double* partials, int nparts, int op, hipStream_t s) {
    hipLaunchKernelGGL(k_scalar, dim3(1), dim3(VT), 0, s, c, partials, nparts, op);
    return hipGetLastError();
}

#define FSD_VEC_INST(T)                                                                          \
    template hipError_t vec_pack<T>(const double*, T*, int, int, long, double, hipStream_t);     \
    template hipError_t vec_unpack<T>(const T*, double*, int, int, long, hipStream_t);           \
    template hipError_t vec_dot<T>(const T*, const T*, long, double*, const Ctrl*, int*,         \
                                   hipStream_t);                                                 \
    template hipError_t vec_update_xr<T>(T*, T*, const T*, const T*, long, const Ctrl*, double*, \
                                         int*, hipStream_t);                                     \
    template hipError_t vec_fill<T>(T*, long, T, hipStream_t);                                   \
    template hipError_t vec_copy<T>(const T*, T*, long, hipStream_t);                            \
    template hipError_t vec_axpy64<T>(double*, const T*, long, double, hipStream_t);            \
    template hipError_t vec_axpy<T>(T*, const T*, long, hipStream_t);

FSD_VEC_INST(double)
FSD_VEC_INST(float)
template hipError_t vec_cast<double, float>(const double*, float*, long, double, hipStream_t);
template hipError_t vec_cast<float, double>(const float*, double*, long, double, hipStream_t);
template hipError_t vec_cast<double, double>(const double*, double*, long, double, hipStream_t);

}  // namespace fsd
