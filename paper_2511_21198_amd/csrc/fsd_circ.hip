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
constexpr int kCircLds = 2048;   // complex line values per workgroup (32 KiB; four workgroups per CU)

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

// buf: lpb lines of M values holding the chirped input (zero beyond n);
// tw: the M/2 twiddles, staged in LDS.  Leaves M times the cyclic
// convolution with the conjugated chirp, natural order.  Two radix-2 stages
// are taken per pass over LDS: the four values j, j + q, j + h, j + h + q
// (decimation in frequency, half sizes h and q = h/2) or j, j + h, j + 2h,
// j + 3h (decimation in time, half sizes h and 2h) are closed under both
// stages, so a thread applies both in registers with the same operations
// as two radix-2 passes; an odd number of stages leaves one radix-2 pass.
__device__ void bluestein_conv(double2* buf, const double2* tw, const CircArgs& a) {
    const int M = a.M, H = M >> 1, logH = a.logM - 1;
    const int Q = M >> 2, nq = a.lpb * Q;
    // forward, decimation in frequency: half sizes h, h/2; twiddle step M / (2h)
    int h = H, lh = logH, ts = 1;
    for (; h >= 2; h >>= 2, lh -= 2, ts <<= 2) {
        const int q = h >> 1, lq = lh - 1;
        for (int b = threadIdx.x; b < nq; b += CT) {
            const int li = b >> (a.logM - 2), r = b & (Q - 1);
            const int g = r >> lq, k = r & (q - 1);
            const int i0 = li * M + 2 * g * h + k;
            const double2 x0 = buf[i0], x1 = buf[i0 + q], x2 = buf[i0 + h], x3 = buf[i0 + h + q];
            const double2 a0 = cadd(x0, x2), a2 = cmul(csub(x0, x2), tw[k * ts]);
            const double2 a1 = cadd(x1, x3), a3 = cmul(csub(x1, x3), tw[(k + q) * ts]);
            const double2 t = tw[k * 2 * ts];
            buf[i0] = cadd(a0, a1);
            buf[i0 + q] = cmul(csub(a0, a1), t);
            buf[i0 + h] = cadd(a2, a3);
            buf[i0 + h + q] = cmul(csub(a2, a3), t);
        }
        __syncthreads();
    }
    if (h == 1) {   // last stage, twiddle 1
        for (int b = threadIdx.x; b < a.lpb * H; b += CT) {
            const int i0 = 2 * b;   // lines are contiguous: pair (2b, 2b + 1)
            const double2 u = buf[i0], v = buf[i0 + 1];
            buf[i0] = cadd(u, v);
            buf[i0 + 1] = csub(u, v);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < a.lpb * M; e += CT) buf[e] = cmul(buf[e], a.bsp[e & (M - 1)]);
    __syncthreads();
    // inverse, decimation in time with conjugate twiddles: half sizes h, 2h
    h = 1;
    lh = 0;
    ts = H;
    for (; 2 * h < M; h <<= 2, lh += 2, ts >>= 2) {
        for (int b = threadIdx.x; b < nq; b += CT) {
            const int li = b >> (a.logM - 2), r = b & (Q - 1);
            const int g = r >> lh, k = r & (h - 1);
            const int i0 = li * M + 4 * g * h + k;
            const double2 x0 = buf[i0], x1 = buf[i0 + h], x2 = buf[i0 + 2 * h], x3 = buf[i0 + 3 * h];
            const double2 t = tw[k * ts];
            const double2 v1 = cmulc(x1, t), v3 = cmulc(x3, t);
            const double2 a0 = cadd(x0, v1), a1 = csub(x0, v1), a2 = cadd(x2, v3), a3 = csub(x2, v3);
            const double2 u2 = cmulc(a2, tw[k * (ts >> 1)]), u3 = cmulc(a3, tw[(k + h) * (ts >> 1)]);
            buf[i0] = cadd(a0, u2);
            buf[i0 + 2 * h] = csub(a0, u2);
            buf[i0 + h] = cadd(a1, u3);
            buf[i0 + 3 * h] = csub(a1, u3);
        }
        __syncthreads();
    }
    if (h < M) {    // last stage, half size M/2
        for (int b = threadIdx.x; b < a.lpb * H; b += CT) {
            const int li = b >> logH, k = b & (H - 1);
            const int i0 = li * M + k;
            const double2 u = buf[i0], v = cmulc(buf[i0 + H], tw[k]);
            buf[i0] = cadd(u, v);
            buf[i0 + H] = csub(u, v);
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
    extern __shared__ double2 lds[];
    if (a.ctrl && a.ctrl->done) return;
    const int M = a.M, n = a.n, lpb = a.lpb;
    double2* tw = lds;             // M/2 twiddles
    double2* buf = lds + M / 2;    // lpb lines of M values
    for (int e = threadIdx.x; e < M / 2; e += CT) tw[e] = a.tw[e];
    // Workgroups go to the 8 XCDs in turn; give each XCD one contiguous run
    // of tiles, so that neighbouring tiles (which share 128-byte lines in
    // the strided passes) meet in one L2.  A bijection on [0, gridDim.x).
    const int nbk = (int)gridDim.x, xq = nbk / 8, xr = nbk % 8;
    const int xcd = (int)blockIdx.x % 8, xi = (int)blockIdx.x / 8;
    const int tile = xcd * xq + min(xcd, xr) + xi;
    const long l0 = (long)tile * lpb;
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
    bluestein_conv(buf, tw, a);
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
        bluestein_conv(buf, tw, a);
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
    const size_t lds = ((size_t)a.lpb * a.M + a.M / 2) * sizeof(double2);
    hipLaunchKernelGGL(k_circ, dim3((unsigned)g), dim3(CT), lds, s, a);
    return hipGetLastError();
}

}  // namespace fsd
