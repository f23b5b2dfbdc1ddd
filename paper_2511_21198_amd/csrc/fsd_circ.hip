// Circulant comparator preconditioners (Section 4): line passes of the
// d-dimensional DFT of lengths n_i with the division by the circulant
// eigenvalues fused into the last axis, float64.
//
// The DFT of a line of length n is Bluestein's chirp transform
//   X_k = w_k sum_j (x_j w_j) conj(w_{k-j}),   w_j = e^{-i pi j^2 / n},
// a convolution taken with FFTs of length M (power of two, M >= 2n - 1) in
// LDS: a decimation-in-frequency FFT (natural order in, bit-reversed out),
// the product with the M-point spectrum of the conjugated chirp (stored in
// bit-reversed order), and a decimation-in-time inverse FFT (bit-reversed in,
// natural out), so no permutation pass is needed.  The inverse DFT is
// conj(DFT(conj X)) / n.  A workgroup holds lpb lines of M complex values;
// the lines of the strided passes are neighbours in x, so each element of
// the lines is one contiguous run of lpb complex values.
#include "fsd_circ.h"

namespace fsd {

namespace {

constexpr int CT = 256;
constexpr int kCircLds = 4096;   // complex values of LDS per workgroup (64 KiB)

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {   // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__device__ inline long line_base(const CircArgs& a, long l) {
    return (l / a.nx) * a.os + (l % a.nx) * a.xs;
}

// buf: lpb lines of M values holding the chirped input (zero beyond n).
// Leaves M times the cyclic convolution with the conjugated chirp, natural
// order.
__device__ void bluestein_conv(double2* buf, const CircArgs& a) {
    const int M = a.M, H = M >> 1, logH = a.logM - 1;
    const int nb = a.lpb * H;
    // forward, decimation in frequency: half size h, twiddle step M / (2h)
    for (int h = H, lh = logH, ts = 1; h >= 1; h >>= 1, --lh, ts <<= 1) {
        for (int b = threadIdx.x; b < nb; b += CT) {
            const int li = b >> logH, r = b & (H - 1);
            const int g = r >> lh, k = r & (h - 1);
            const int i0 = li * M + 2 * g * h + k, i1 = i0 + h;
            const double2 u = buf[i0], v = buf[i1];
            buf[i0] = cadd(u, v);
            buf[i1] = cmul(csub(u, v), a.tw[k * ts]);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < a.lpb * M; e += CT) buf[e] = cmul(buf[e], a.bsp[e & (M - 1)]);
    __syncthreads();
    // inverse, decimation in time with conjugate twiddles
    for (int h = 1, lh = 0, ts = H; h < M; h <<= 1, ++lh, ts >>= 1) {
        for (int b = threadIdx.x; b < nb; b += CT) {
            const int li = b >> logH, r = b & (H - 1);
            const int g = r >> lh, k = r & (h - 1);
            const int i0 = li * M + 2 * g * h + k, i1 = i0 + h;
            const double2 u = buf[i0], v = cmulc(buf[i1], a.tw[k * ts]);
            buf[i0] = cadd(u, v);
            buf[i1] = csub(u, v);
        }
        __syncthreads();
    }
}

// Element (line li, position j) of the e-th work item: lines along x
// (stride 1) take j fastest, strided lines take the line fastest.
__device__ inline void item(const CircArgs& a, int e, int span, int& li, int& j) {
    if (a.st == 1) {
        li = e / span;
        j = e - li * span;
    } else {
        j = e / a.lpb;
        li = e - j * a.lpb;
    }
}

__global__ __launch_bounds__(CT) void k_circ(CircArgs a) {
    extern __shared__ double2 buf[];
    if (a.ctrl && a.ctrl->done) return;
    const int M = a.M, n = a.n, lpb = a.lpb;
    const long l0 = (long)blockIdx.x * lpb;
    const int nl = (int)min((long)lpb, a.nlines - l0);
    const bool inv_in = a.mode == CM_INV || a.mode == CM_INV_C2R;
    const bool inv_out = a.mode != CM_FWD_R2C && a.mode != CM_FWD;

    for (int e = threadIdx.x; e < lpb * M; e += CT) {
        int li, j;
        item(a, e, M, li, j);
        double2 v = make_double2(0.0, 0.0);
        if (li < nl && j < n) {
            const long g = line_base(a, l0 + li) + (long)j * a.st;
            v = a.mode == CM_FWD_R2C ? make_double2(a.in_r[g], 0.0) : a.in_c[g];
            if (inv_in) v.y = -v.y;
            v = cmul(v, a.w[j]);
        }
        buf[li * M + j] = v;
    }
    __syncthreads();
    bluestein_conv(buf, a);
    const double sM = 1.0 / M;

    if (a.mode == CM_LAST) {
        // X_k = w_k y_k / M, then X / Lambda, conjugated and chirped as the
        // input of the inverse transform
        for (int e = threadIdx.x; e < lpb * M; e += CT) {
            const int li = e / M, k = e - li * M;
            double2 v = make_double2(0.0, 0.0);
            if (li < nl && k < n) {
                double2 X = cmul(buf[e], a.w[k]);
                X.x *= sM;
                X.y *= sM;
                const long l = l0 + li;
                const int x = (int)(l % a.nx);
                const int o = (int)(l / a.nx);
                const double2 a1 = a.ea[0][x], b1 = a.eb[0][x];
                double2 lam;
                if (a.dim == 3) {
                    const double2 a2 = a.ea[1][o], b2 = a.eb[1][o];
                    const double2 a3 = a.ea[2][k], b3 = a.eb[2][k];
                    lam = cadd(cmul(a3, cadd(cmul(a2, cadd(a1, b1)), cmul(b2, a1))),
                               cmul(b3, cmul(a2, a1)));
                } else {
                    const double2 a2 = a.ea[1][k], b2 = a.eb[1][k];
                    lam = cadd(cmul(a2, cadd(a1, b1)), cmul(b2, a1));
                }
                const double den = lam.x * lam.x + lam.y * lam.y;
                double2 q = cmulc(X, lam);
                q.x /= den;
                q.y = -q.y / den;
                v = cmul(q, a.w[k]);
            }
            buf[e] = v;
        }
        __syncthreads();
        bluestein_conv(buf, a);
    }

    const double sc = inv_out ? sM / n : sM;
    for (int e = threadIdx.x; e < lpb * M; e += CT) {
        int li, j;
        item(a, e, M, li, j);
        if (li < nl && j < n) {
            double2 X = cmul(buf[li * M + j], a.w[j]);
            X.x *= sc;
            X.y *= inv_out ? -sc : sc;
            const long g = line_base(a, l0 + li) + (long)j * a.st;
            if (a.mode == CM_INV_C2R) a.out_r[g] = X.x;
            else a.out_c[g] = X;
        }
    }
    if (a.mode == CM_INV_C2R && a.pad > n) {   // zero padding columns (x lines, stride 1)
        const int zw = a.pad - n;
        for (int e = threadIdx.x; e < lpb * zw; e += CT) {
            const int li = e / zw, j = n + (e - li * zw);
            if (li < nl) a.out_r[line_base(a, l0 + li) + j] = 0.0;
        }
    }
}

}  // namespace

int circ_lines_per_block(int M) {
    int lpb = kCircLds / M;
    if (lpb > 64) lpb = 64;
    return lpb < 1 ? 1 : lpb;
}

hipError_t launch_circ(const CircArgs& a, hipStream_t s) {
    if (a.M < 2 || (a.M & (a.M - 1)) != 0 || (1 << a.logM) != a.M || a.M < 2 * a.n - 1 ||
        a.lpb < 1 || a.lpb * a.M > kCircLds || a.nx < 1 || a.n < 1)
        return hipErrorInvalidValue;
    if (a.mode == CM_INV_C2R && a.pad > a.n && a.st != 1) return hipErrorInvalidValue;
    if (a.nlines <= 0) return hipSuccess;
    const long g = (a.nlines + a.lpb - 1) / a.lpb;
    const size_t lds = (size_t)a.lpb * a.M * sizeof(double2);
    hipLaunchKernelGGL(k_circ, dim3((unsigned)g), dim3(CT), lds, s, a);
    return hipGetLastError();
}

}  // namespace fsd
