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

// First residual of a CN step from the previous state (x0 = u^{m-1}):
// b = (A_N - K) u + dt F and A u = (A_N + K) u give
// r = b - A u = 2 (b - A_N u) - dt F, with A_N = A_{n3} (x) A_{n2} (x) A_{n1}
// the separable tridiagonal mass operator (1, 6, 1)/8 per axis (zero beyond
// the boundary; Section 2, ``linear_sys``): a 27-point stencil (9-point in
// 2D, A_N = A_{n2} (x) A_{n1}) instead of a Toeplitz matvec.  Padded layout
// [n3][n2][P1] (n3 = 1 in 2D); F dense [n3][n2][n1] (may be null: f = 0);
// padding columns of r are written as zeros.  Partial ||r||^2.
// One wave owns a tile of 64 columns x kRpY rows x rz planes and marches
// through its planes, keeping the (y, x)-filtered values of three
// consecutive planes in registers; the x neighbours are two more loads of
// the same cache lines.  u is read once from HBM (the halo rows and planes
// of a tile come from the caches), b and F once, r written once.
constexpr int kRpY = 8, kRpZ = 16;   // rows per tile; planes per tile at most (rz <= kRpZ)

// s[i] = (A_{n2} (x) A_{n1} u)(y0 + i) on plane zz (zero outside the grid).
// Loads are branch-free: indices are clamped into the grid and values
// outside it replaced by zero, so all loads of a plane issue together.
__device__ inline void resid_plane(const double* __restrict__ u, int xl, int xm, int xp, bool inx,
                                   bool hasm, bool hasp, int n2, int n3, int P1, int y0, int zz,
                                   double (&s)[kRpY]) {
    if (zz < 0 || zz >= n3) {   // uniform: a plane beyond the grid
#pragma unroll
        for (int i = 0; i < kRpY; ++i) s[i] = 0.0;
        return;
    }
    double h[kRpY + 2];
#pragma unroll
    for (int j = 0; j < kRpY + 2; ++j) {
        const int yy = y0 - 1 + j;
        const int yc = yy < 0 ? 0 : (yy >= n2 ? n2 - 1 : yy);
        const double* ur = u + ((long)zz * n2 + yc) * P1;
        const double c = ur[xl], m = ur[xm], p = ur[xp];
        const double v = 0.75 * c + 0.125 * (hasm ? m : 0.0) + 0.125 * (hasp ? p : 0.0);
        h[j] = (inx && yy >= 0 && yy < n2) ? v : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kRpY; ++i) s[i] = 0.125 * h[i] + 0.75 * h[i + 1] + 0.125 * h[i + 2];
}

__global__ __launch_bounds__(VT) void k_resid_prev(const double* __restrict__ u,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ F, double* __restrict__ r,
                                                   int n1, int n2, int n3, int P1, int dim, int rz,
                                                   double dt, double* __restrict__ partials) {
    __shared__ double sb[VT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nxc = (P1 + 63) / 64, nyc = (n2 + kRpY - 1) / kRpY, nzc = (n3 + rz - 1) / rz;
    const long nwt = (long)nxc * nyc * nzc;
    const double wc = dim == 2 ? 1.0 : 0.75;   // 2D: no z factor (planes -1 and 1 are empty)
    double acc = 0.0;
    for (long t = (long)blockIdx.x * (VT / 64) + wid; t < nwt; t += (long)gridDim.x * (VT / 64)) {
        const int xc = (int)(t % nxc);
        const long t2 = t / nxc;
        const int y0 = (int)(t2 % nyc) * kRpY, z0 = (int)(t2 / nyc) * rz;
        const int x = xc * 64 + lane;
        const bool inx = x < n1, inp = x < P1;
        // clamped columns: every load stays inside the row
        const int xl = x < P1 ? x : P1 - 1, xm = xl > 0 ? xl - 1 : 0, xp = xl + 1 < P1 ? xl + 1 : xl;
        const int xf = x < n1 ? x : n1 - 1;
        const bool hasm = x > 0, hasp = x + 1 < n1;
        double sm[kRpY], sc[kRpY], sp[kRpY];
        resid_plane(u, xl, xm, xp, inx, hasm, hasp, n2, n3, P1, y0, z0 - 1, sm);
        resid_plane(u, xl, xm, xp, inx, hasm, hasp, n2, n3, P1, y0, z0, sc);
        for (int k = 0; k < rz && z0 + k < n3; ++k) {
            const int z = z0 + k;
            resid_plane(u, xl, xm, xp, inx, hasm, hasp, n2, n3, P1, y0, z + 1, sp);
#pragma unroll
            for (int i = 0; i < kRpY; ++i) {
                const int y = y0 + i;
                if (y < n2) {   // uniform
                    const long row = (long)z * n2 + y;
                    const double bv = b[row * P1 + xl];
                    const double fv = F ? F[xf + (long)n1 * row] : 0.0;
                    const double an = 0.125 * sm[i] + wc * sc[i] + 0.125 * sp[i];
                    const double v = inx ? 2.0 * (bv - an) - dt * fv : 0.0;
                    if (inp) r[row * P1 + x] = v;
                    acc += v * v;
                }
                sm[i] = sc[i];
                sc[i] = sp[i];
            }
        }
    }
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

// Streaming copy of n 16-byte words: each workgroup copies one contiguous
// chunk of kCopyChunk words, eight loads in flight per thread before the
// non-temporal stores.  Measured on an MI355X (1 GiB): 5.35 TB/s read +
// write, against 4.3-5.1 TB/s for grid-stride variants and 5.2 TB/s for
// hipMemcpy device to device.
constexpr long kCopyChunk = 16384;
typedef unsigned int cp_u4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(VT) void k_stream_copy(const cp_u4* __restrict__ a,
                                                    cp_u4* __restrict__ b, long n) {
    const long beg = blockIdx.x * kCopyChunk;
    const long end = beg + kCopyChunk < n ? beg + kCopyChunk : n;
    for (long e = beg + threadIdx.x; e < end; e += 8 * VT) {
        cp_u4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const long i = e + k * VT;
            v[k] = i < end ? a[i] : cp_u4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const long i = e + k * VT;
            if (i < end) __builtin_nontemporal_store(v[k], b + i);
        }
    }
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
// then the Krylov scalar update selected by op.  1024 threads, four loads in
// flight per thread: the partials of a strided pass number a few thousand.
constexpr int SVT = 1024;
__global__ __launch_bounds__(SVT) void k_scalar(Ctrl* c, const double* __restrict__ partials,
                                                int nparts, int op) {
    __shared__ double sb[SVT / 64];
    if (c->done) return;
    double acc = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < nparts; i += SVT) acc += partials[i];
    acc = wave_sum(acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sb[w] = acc;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double S = 0.0;
#pragma unroll
    for (int i = 0; i < SVT / 64; ++i) S += sb[i];
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
        case SC_STORE_BB:
            c->bb = S;
            break;
        case SC_STORE_RZ:
            c->rz = S;
            break;
        case SC_STORE_RR:
            c->rr = S;
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
hipError_t resid_prev(const double* u, const double* b, const double* F, double* r, int n1, int n2,
                      int n3, int P1, int dim, double dt, double* partials, int* nparts,
                      hipStream_t s) {
    // planes per tile: 16 (255^3: 206 us against 218 with 8, fewer halo
    // planes read again), halved while the grid has fewer than 2048 wave
    // tiles (small grids would leave most of the chip idle)
    const long nxy = (long)((P1 + 63) / 64) * ((n2 + kRpY - 1) / kRpY);
    int rz = kRpZ;
    while (rz > 1 && nxy * ((n3 + rz - 1) / rz) < 2048) rz >>= 1;
    const long nwt = nxy * ((n3 + rz - 1) / rz);
    const int g = (int)std::max(1L, std::min<long>((nwt + VT / 64 - 1) / (VT / 64), kVecGrid));
    *nparts = g;
    hipLaunchKernelGGL(k_resid_prev, dim3(g), dim3(VT), 0, s, u, b, F, r, n1, n2, n3, P1, dim, rz, dt,
                       partials);
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
hipError_t stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const long n = (long)(bytes / 16);
    if (n == 0) return hipSuccess;
    const long g = (n + kCopyChunk - 1) / kCopyChunk;
    if (g > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)g), dim3(VT), 0, s,
                       reinterpret_cast<const cp_u4*>(src), reinterpret_cast<cp_u4*>(dst), n);
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
    hipLaunchKernelGGL(k_scalar, dim3(1), dim3(SVT), 0, s, c, partials, nparts, op);
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
