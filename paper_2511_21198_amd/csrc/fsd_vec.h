// Host launchers of the vector / reduction / scalar kernels (fsd_vec.hip).
#pragma once

#include "fsd_internal.h"

namespace fsd {

// Fixed reduction grid: vector kernels use at most this many workgroups, so
// the number of partial sums (and their summation order) depends only on N.
constexpr int kVecGrid = 1024;

// Scalar-kernel operations (see k_scalar).
enum ScalarOp : int {
    SC_BB = 0,     // bb = S, thresh = tol^2 bb
    SC_RR0 = 1,    // rr = S, done if rr <= thresh
    SC_RZ0 = 2,    // rz = S, first = 1
    SC_ALPHA = 3,  // pq = S, alpha = rz / pq (breakdown if pq <= 0)
    SC_CHECK = 4,  // rr = S, iters += 1, done if rr <= thresh or iters >= maxit
    SC_BETA = 5,   // beta = S / rz, rz = S, first = 0
    SC_STORE = 6,  // pq = S (plain reduction result for the host)
    SC_STORE_BB = 7,  // bb = S (a second plain result, read with the first)
    SC_STORE_RZ = 8,  // rz = S (a third one)
    SC_STORE_RR = 9,  // rr = S (a fourth one)
};

int vec_grid(long N);

template <typename T>
hipError_t vec_pack(const double* dense, T* pad, int n1, int P1, long rows, double scale, hipStream_t s);
template <typename T>
hipError_t vec_unpack(const T* pad, double* dense, int n1, int P1, long rows, hipStream_t s);
template <typename T>
hipError_t vec_dot(const T* a, const T* b, long N, double* partials, const Ctrl* ctrl, int* nparts,
                   hipStream_t s);
template <typename T>
hipError_t vec_update_xr(T* x, T* r, const T* p, const T* q, long N, const Ctrl* ctrl,
                         double* partials, int* nparts, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t vec_cast(const Tin* in, Tout* out, long N, double scale, hipStream_t s);
template <typename Td>
hipError_t vec_axpy64(double* x, const Td* d, long N, double scale, hipStream_t s);
template <typename T>
hipError_t vec_axpy(T* x, const T* d, long N, hipStream_t s);   // x += d
// r = b - A u^{m-1} for b = rhs(u^{m-1}, F): 2 (b - A_N u) - dt F, partial ||r||^2
hipError_t resid_prev(const double* u, const double* b, const double* F, double* r, int n1, int n2,
                      int n3, int P1, int dim, double dt, double* partials, int* nparts,
                      hipStream_t s);
template <typename T>
hipError_t vec_fill(T* x, long N, T v, hipStream_t s);
template <typename T>
hipError_t vec_copy(const T* a, T* b, long N, hipStream_t s);
// Streaming copy of bytes (a multiple of 16; 16-byte aligned pointers).
hipError_t stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// have != 0: x <- 2 x - up and up <- old x; have == 0: up <- x.
hipError_t vec_extrap(double* x, double* up, long N, int have, hipStream_t s);
// abs2: absolute floor of the stopping threshold, thresh = max(tol2 bb, abs2).
hipError_t ctrl_init(Ctrl* c, double tol2, int maxit, int restart, hipStream_t s,
                     double abs2 = 0.0, double eta2 = 0.5);
hipError_t scalar_step(Ctrl* c, const double* partials, int nparts, int op, hipStream_t s);

}  // namespace fsd
