// Column engine for the float32 strided (y / z) passes of length L = 512
// (n = 255): the transforms of a tile's lines are split between threads by
// residue, so that global loads and stores go straight between registers and
// HBM rows, and one LDS transpose per transform is the only data exchange.
//
// Tile: CP = 16 complex lines (x positions x0 + 2p and x0 + 2p + 1 packed as
// real and imaginary parts, a 128-byte row segment) at one outer index;
// 256 threads, thread (p, r) with p = tid % 16 and r = tid / 16.
//
// Forward transform of a line V of length L = 512 = 16 x 32 (Cooley-Tukey,
// j = r + 16 m, k = k1 + 32 k2):
//   X[k1 + 32 k2] = sum_r w16^{r k2} (w512^{r k1} sum_m V[r + 16 m] w32^{m k1}).
// Thread (p, r) holds V[r + 16 m] for its residue r (the rows r + 16 m of
// the grid), computes the 32-point DFTs over m and the twiddles in
// registers, and the tile is transposed through LDS so that thread (p, t)
// holds the columns k1 = t and t + 16, whose 16-point DFTs over r give
// X[k1 + 32 k2].  A second forward transform of a spectrum held that way
// (j = j1 + 16 j2, inputs f = k1 + 32 k2) runs the same steps in the other
// order and leaves Y[j1 + 16 j2] in thread (p, j1): the rows it read.
//
// LDS: the transpose runs in two halves of k1 through a 32 KB buffer, plus
// the twiddle table (4 KB), so four workgroups fit on a CU.
#pragma once

#include <type_traits>

#include "fsd_wave.hpp"

namespace fsd {
namespace colx {

constexpr int L = 512;          // transform length
constexpr int NN = L / 2 - 1;   // line length n
constexpr int CR = 16;          // residues: threads per complex line
constexpr int CP = 16;          // complex lines per tile
constexpr int NT = CR * CP;     // threads per workgroup
constexpr int TX = 2 * CP;      // x positions per tile

// cos(2 pi q / 32) for q = 0..8
__host__ __device__ constexpr float c32base(int q) {
    return q == 0 ? 1.0f : q == 1 ? 0.98078528040323044913f : q == 2 ? 0.92387953251128675613f
         : q == 3 ? 0.83146961230254523708f : q == 4 ? 0.70710678118654752440f
         : q == 5 ? 0.55557023301960222474f : q == 6 ? 0.38268343236508977173f
         : q == 7 ? 0.19509032201612826785f : 0.0f;
}
__host__ __device__ constexpr float cos32(int q) {
    q &= 31;
    return q <= 8 ? c32base(q) : q <= 16 ? -c32base(16 - q) : q <= 24 ? -c32base(q - 16)
                                                                       : c32base(32 - q);
}
__host__ __device__ constexpr float sin32(int q) { return cos32(q - 8); }

template <int B, int E, typename F>
__device__ inline void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// x *= w32^Q, w32 = exp(-2 pi i / 32)
template <int Q>
__device__ inline void mul_w32(float& xr, float& xi) {
    constexpr int q = Q & 31;
    if constexpr (q == 0) {
        return;
    } else if constexpr (q == 8) {          // -i
        const float t = xr; xr = xi; xi = -t;
    } else if constexpr (q == 16) {
        xr = -xr; xi = -xi;
    } else if constexpr (q == 24) {         // +i
        const float t = xr; xr = -xi; xi = t;
    } else {
        constexpr float c = cos32(q), s = sin32(q);
        const float a = xr, b = xi;
        xr = a * c + b * s;
        xi = b * c - a * s;
    }
}

// 32-point forward DFT in registers (n = 4 n1 + n2, k = k1 + 8 k2).
// NOUT = 16: only outputs 0..15 are needed.
template <int NOUT = 32>
__device__ inline void dft32(float (&xr)[32], float (&xi)[32]) {
    float tr[4][8], ti[4][8];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) {
            tr[n2][n1] = xr[4 * n1 + n2];
            ti[n2][n1] = xi[4 * n1 + n2];
        }
        dft8(tr[n2], ti[n2]);
    }
    static_for<1, 8>([&](auto K) {
        constexpr int k = decltype(K)::value;
        mul_w32<k>(tr[1][k], ti[1][k]);
        mul_w32<2 * k>(tr[2][k], ti[2][k]);
        mul_w32<3 * k>(tr[3][k], ti[3][k]);
    });
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
        const float a0r = tr[0][k1], a0i = ti[0][k1], a1r = tr[1][k1], a1i = ti[1][k1];
        const float a2r = tr[2][k1], a2i = ti[2][k1], a3r = tr[3][k1], a3i = ti[3][k1];
        const float s02r = a0r + a2r, s02i = a0i + a2i, d02r = a0r - a2r, d02i = a0i - a2i;
        const float s13r = a1r + a3r, s13i = a1i + a3i, d13r = a1r - a3r, d13i = a1i - a3i;
        xr[k1] = s02r + s13r;       xi[k1] = s02i + s13i;
        xr[k1 + 8] = d02r + d13i;   xi[k1 + 8] = d02i - d13r;
        if constexpr (NOUT == 32) {
            xr[k1 + 16] = s02r - s13r;  xi[k1 + 16] = s02i - s13i;
            xr[k1 + 24] = d02r - d13i;  xi[k1 + 24] = d02i + d13r;
        }
    }
}

// 16-point forward DFT (n = 4 n1 + n2, k = k1 + 4 k2), in place; NOUT = 8:
// only outputs 0..7 are needed.
template <int NOUT = 16>
__device__ inline void dft16(float (&xr)[16], float (&xi)[16]) {
    float ar[4][4], ai[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
            ar[n2][n1] = xr[4 * n1 + n2];
            ai[n2][n1] = xi[4 * n1 + n2];
        }
        dft4(ar[n2], ai[n2]);
    }
    static_for<1, 4>([&](auto K) {
        constexpr int k = decltype(K)::value;
        mul_w32<2 * k>(ar[1][k], ai[1][k]);
        mul_w32<4 * k>(ar[2][k], ai[2][k]);
        mul_w32<6 * k>(ar[3][k], ai[3][k]);
    });
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        const float a0r = ar[0][k1], a0i = ai[0][k1], a1r = ar[1][k1], a1i = ai[1][k1];
        const float a2r = ar[2][k1], a2i = ai[2][k1], a3r = ar[3][k1], a3i = ai[3][k1];
        const float s02r = a0r + a2r, s02i = a0i + a2i, d02r = a0r - a2r, d02i = a0i - a2i;
        const float s13r = a1r + a3r, s13i = a1i + a3i, d13r = a1r - a3r, d13i = a1i - a3i;
        xr[k1] = s02r + s13r;      xi[k1] = s02i + s13i;
        xr[k1 + 4] = d02r + d13i;  xi[k1 + 4] = d02i - d13r;
        if constexpr (NOUT == 16) {
            xr[k1 + 8] = s02r - s13r;   xi[k1 + 8] = s02i - s13i;
            xr[k1 + 12] = d02r - d13i;  xi[k1 + 12] = d02i + d13r;
        }
    }
}

struct Smem {
    float2 buf[16 * CR * CP];   // half a transpose (also the mirror exchange)
    float2 tw[L];               // exp(-2 pi i e / L)
};

struct Tile {
    int p, r;
    long base;     // element offset of (x0 + 2p, row 0) at the tile's outer index
    bool pad0, pad1;
};

__device__ inline Tile tile_of(const PassGeo& g) {
    Tile t;
    const int tid = threadIdx.x;
    t.p = tid & (CP - 1);
    t.r = tid >> 4;
    const int ntx = g.P1 / TX;
    const int xt = blockIdx.x % ntx, o = blockIdx.x / ntx;
    const int x = xt * TX + 2 * t.p;
    t.base = (long)o * g.ostride + x;
    t.pad0 = x >= g.nx;
    t.pad1 = x + 1 >= g.nx;
    return t;
}

// Table of L values into LDS, L / NT per thread.  The trip count is a
// constant and the loop unrolled, so every load of a thread is issued
// before the first LDS store (a loop over threadIdx.x would wait for each
// load in turn at the start of every workgroup).
__device__ inline void stage_table(float2* dst, const float* __restrict__ src) {
    static_assert(L % NT == 0, "table length");
    float2 v[L / NT];
#pragma unroll
    for (int k = 0; k < L / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        v[k] = make_float2(src[2 * e], src[2 * e + 1]);
    }
#pragma unroll
    for (int k = 0; k < L / NT; ++k) dst[threadIdx.x + k * NT] = v[k];
}

__device__ inline void load_tw(Smem& S, const float* __restrict__ tw) { stage_table(S.tw, tw); }

__device__ inline const float2* row2(const float* v, long off) {
    return reinterpret_cast<const float2*>(v + off);
}
__device__ inline float2* row2(float* v, long off) { return reinterpret_cast<float2*>(v + off); }

// Points r + 16 m (m = 0..31) of the odd extensions (V[0] = V[n+1] = 0,
// V[j] = u[j-1], V[L-j] = -V[j]) of the tile's two real lines per complex
// line.  The mirrored half comes from thread (p, 16 - r) through LDS.
// Ends with the LDS buffer free (barrier).
__device__ inline void load_odd(Smem& S, const Tile& t, const float* __restrict__ u, long es,
                                float (&xr)[32], float (&xi)[32]) {
    float2 v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int j = t.r + 16 * m;   // <= n
        v[m] = j >= 1 ? *row2(u, t.base + (long)(j - 1) * es) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        S.buf[(t.r * 16 + m) * CP + t.p] = v[m];
        xr[m] = v[m].x;
        xi[m] = v[m].y;
    }
    __syncthreads();
    const int rp = (16 - t.r) & 15;
#pragma unroll
    for (int m = 16; m < 32; ++m) {
        // V[r + 16 m] = -V[(16 - r) + 16 (31 - m)] (r >= 1), -V[16 (32 - m)] (r = 0)
        float2 w;
        if (t.r == 0) {
            const int mm = 32 - m;
            w = mm == 16 ? make_float2(0.f, 0.f) : S.buf[mm * CP + t.p];
        } else {
            w = S.buf[(rp * 16 + (31 - m)) * CP + t.p];
        }
        xr[m] = -w.x;
        xi[m] = -w.y;
    }
    __syncthreads();
}

// After the per-thread 32-point DFTs (B[k1] in xr/xi), half h of the
// transpose: y[rr] = w512^{rr k1} B_rr[k1] for k1 = t + 16 h, gathered from
// the 16 residues rr (reads xr[16 h .. 16 h + 15] only).
__device__ inline void transpose_fwd_half(Smem& S, const Tile& t, int h, const float (&xr)[32],
                                          const float (&xi)[32], float (&yr)[16], float (&yi)[16]) {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        const int k1 = kk + 16 * h;
        const float2 w = S.tw[t.r * k1];
        const float a = xr[k1], b = xi[k1];
        S.buf[(kk * CR + t.r) * CP + t.p] = make_float2(a * w.x - b * w.y, a * w.y + b * w.x);
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < CR; ++rr) {
        const float2 w = S.buf[(t.r * CR + rr) * CP + t.p];
        yr[rr] = w.x;
        yi[rr] = w.y;
    }
    __syncthreads();
}

// Second transform, half h: thread (p, t) holds the spectrum at
// f = k1 + 32 k2 (k1 = t + 16 h) after its 16-point DFTs over k2 (outputs j1);
// scales them by the twiddles w512^{k1 j1} and gathers, for j1 = r, the
// values of the 16 columns k1 of this half into xr[16 h .. 16 h + 15].
__device__ inline void transpose_inv_half(Smem& S, const Tile& t, int h, const float (&dr)[16],
                                          const float (&di)[16], float (&xr)[32], float (&xi)[32]) {
    const int k1 = t.r + 16 * h;
#pragma unroll
    for (int j1 = 0; j1 < 16; ++j1) {
        const float2 w = S.tw[k1 * j1];
        const float a = dr[j1], b = di[j1];
        S.buf[(j1 * CR + t.r) * CP + t.p] = make_float2(a * w.x - b * w.y, a * w.y + b * w.x);
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < CR; ++tt) {
        const float2 w = S.buf[(t.r * CR + tt) * CP + t.p];
        xr[tt + 16 * h] = w.x;
        xi[tt + 16 * h] = w.y;
    }
    __syncthreads();
}

// Strided DST-I pass (SCALE = false), or the last-axis pass S Lambda^{-1} S
// with the Parseval partials of (r, P^{-1} r) (SCALE = true).
// Register budget: four wavefronts per SIMD (128 VGPRs) for the plain pass;
// the scale pass holds both halves of a transpose plus the Lambda operands
// and is compiled for three (168 VGPRs) instead of spilling.
template <bool SCALE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(SCALE ? 3 : 4)))
void k_col_dst(DstArgs<float> a) {
    __shared__ Smem S;
    __shared__ double s_red[NT / 64];
    if (a.ctrl && a.ctrl->done) return;
    const Tile t = tile_of(a.g);
    const long es = a.g.estride;
    load_tw(S, a.tw);
    float xr[32], xi[32];
    load_odd(S, t, a.u, es, xr, xi);
    dft32(xr, xi);
    float yr[2][16], yi[2][16];
    if constexpr (!SCALE) {
        transpose_fwd_half(S, t, 0, xr, xi, yr[0], yi[0]);
        transpose_fwd_half(S, t, 1, xr, xi, yr[1], yi[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k1 = t.r + 16 * h;
            dft16<8>(yr[h], yi[h]);
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) {
                const int k = k1 + 32 * k2;   // DST index 1..n -> row k - 1
                if (k >= 1) {
                    const float s0 = t.pad0 ? 0.f : -yi[h][k2] * a.c;
                    const float s1 = t.pad1 ? 0.f : yr[h][k2] * a.c;
                    st_nt2(a.o + t.base + (long)(k - 1) * es, s0, s1);
                }
            }
        }
    } else {
        // Lambda on line x at frequency k: a_last[k] P(x) + lc_last[k] Q(x)
        float P[2], Q[2];
        {
            const int o = blockIdx.x / (a.g.P1 / TX);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int x = (int)(t.base - (long)o * a.g.ostride) + c;
                P[c] = 0.f;
                Q[c] = 0.f;
                if (x < a.g.nx) {
                    const float a1 = a.a1[x], l1 = a.lc1[x];
                    if (a.dim == 2) {
                        P[c] = a1 + l1;
                        Q[c] = a1;
                    } else {
                        const float a2 = a.a2[o], l2 = a.lc2[o];
                        P[c] = a2 * (a1 + l1) + l2 * a1;
                        Q[c] = a2 * a1;
                    }
                }
            }
        }
        double acc = 0.0;
        // each half of k1: 16-point DFTs over r (spectrum at f = k1 + 32 k2),
        // the Lambda^{-1} scale, 16-point DFTs over k2, then its half of the
        // second transpose
        transpose_fwd_half(S, t, 0, xr, xi, yr[0], yi[0]);
        transpose_fwd_half(S, t, 1, xr, xi, yr[1], yi[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k1 = t.r + 16 * h;
            dft16<16>(yr[h], yi[h]);
#pragma unroll
            for (int k2 = 0; k2 < 16; ++k2) {
                const int f = k1 + 32 * k2;
                const int k = f <= NN ? f : L - f;
                float wr = 0.f, wi = 0.f;
                if (k >= 1 && k <= NN) {
                    const float ak = a.a_last[k - 1], lk = a.lc_last[k - 1];
                    const float inv0 = P[0] != 0.f ? lam_inv(ak * P[0] + lk * Q[0], a.half) : 0.f;
                    const float inv1 = P[1] != 0.f ? lam_inv(ak * P[1] + lk * Q[1], a.half) : 0.f;
                    const float s1 = -yi[h][k2] * a.c;
                    const float s2 = yr[h][k2] * a.c;
                    wr = s1 * inv0;
                    wi = s2 * inv1;
                    if (f <= NN) acc += (double)s1 * (double)wr + (double)s2 * (double)wi;
                }
                yr[h][k2] = wr;
                yi[h][k2] = wi;
            }
            dft16<16>(yr[h], yi[h]);
            transpose_inv_half(S, t, h, yr[h], yi[h], xr, xi);
        }
        dft32<16>(xr, xi);
#pragma unroll
        for (int j2 = 0; j2 < 16; ++j2) {
            const int j = t.r + 16 * j2;   // DST index 1..n -> row j - 1
            if (j >= 1) {
                const float s0 = t.pad0 ? 0.f : -xi[j2] * a.c;
                const float s1 = t.pad1 ? 0.f : xr[j2] * a.c;
                st_nt2(a.o + t.base + (long)(j - 1) * es, s0, s1);
            }
        }
        if (a.partials) {
            const double s = block_sum<NT>(acc, s_red);
            if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
        }
    }
}

// ------------------------------------------------- half-length DST-I
// The unnormalised DST-I of order n = 255, S_k = sum_{j=1}^{255} x_j
// sin(pi j k / N) with N = n + 1 = 256, from one complex FFT of length N
// instead of 2N (the odd extension): with x_0 = x_N = 0 and
//   y_j = sin(pi j / N) (x_j + x_{N-j}) + (x_j - x_{N-j}) / 2,
// the DFT Y_f = sum_j y_j e^{-2 pi i j f / N} = C_f - i D_f gives
//   S_{2f} = D_f  and  S_{2f+1} - S_{2f-1} = C_f  (S_{-1} = -S_1),
// the odd outputs by a prefix sum.  Two real lines share the complex FFT
// (real and imaginary parts of y) and are separated by the symmetry of a
// real sequence's DFT, Y1_f = (Z_f + conj Z_{N-f}) / 2 and
// Y2_f = (Z_f - conj Z_{N-f}) / (2i).  The FFT of length 256 = 16 x 16 runs
// as the column engine's length-512 transform does: 16-point DFTs over m
// in registers (thread (p, r) holds points r + 16 m), the twiddles
// w256^{r k1}, one LDS transpose, 16-point DFTs over r.
constexpr int HN = 256;

// Forward DFT of length 256: on entry thread (p, r) holds z[r + 16 m] in
// (zr[m], zi[m]); on exit Z[r + 16 k2] in (zr[k2], zi[k2]).
__device__ inline void fft256_cols(Smem& S, const Tile& t, float (&zr)[16], float (&zi)[16]) {
    dft16<16>(zr, zi);   // B_r[k1] over m
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) {
        const float2 w = S.tw[2 * t.r * k1];   // w256^{r k1} = w512^{2 r k1}
        const float a = zr[k1], b = zi[k1];
        S.buf[(k1 * CR + t.r) * CP + t.p] = make_float2(a * w.x - b * w.y, a * w.y + b * w.x);
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < CR; ++rr) {
        const float2 v = S.buf[(t.r * CR + rr) * CP + t.p];
        zr[rr] = v.x;
        zi[rr] = v.y;
    }
    __syncthreads();
    dft16<16>(zr, zi);   // over r: Z[k1 + 16 k2] with k1 = r
}

// Unnormalised DST-I of the tile's line pairs.  On entry S.buf[j * CP + p]
// holds x_j for j = 0..255 (x_0 = 0) and a barrier has passed; on exit
// thread (p, t) holds S_k for k = 16 t + q in (sr[q], si[q]), q = 0..15
// (the real-part line in sr, the imaginary-part line in si; k = 0 gives 0),
// and the LDS buffer is free.  tot: 16 * CP float2 of LDS.
__device__ inline void dst256_from_lds(Smem& S, float2* tot, const Tile& t, float (&sr)[16],
                                       float (&si)[16]) {
    float zr[16], zi[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int j = t.r + 16 * m;
        const float2 x = S.buf[j * CP + t.p];
        const float2 xm = S.buf[((HN - j) & (HN - 1)) * CP + t.p];   // x_{N-j} (x_N = x_0 = 0)
        const float sn = -S.tw[j].y;                                  // sin(pi j / N)
        zr[m] = sn * (x.x + xm.x) + 0.5f * (x.x - xm.x);
        zi[m] = sn * (x.y + xm.y) + 0.5f * (x.y - xm.y);
    }
    __syncthreads();
    fft256_cols(S, t, zr, zi);
    // Z_f for f = t + 16 k2 in natural order, then Z_{N-f}
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) S.buf[(t.r + 16 * k2) * CP + t.p] = make_float2(zr[k2], zi[k2]);
    __syncthreads();
    float br[8], bi[8];
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const int f = t.r + 16 * k2;
        const float2 v = S.buf[((HN - f) & (HN - 1)) * CP + t.p];
        br[k2] = v.x;
        bi[k2] = v.y;
    }
    __syncthreads();
    // f < 128: C (both lines) to rows 0..127 of the buffer, D to rows 128..255
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const int f = t.r + 16 * k2;
        const float ar = zr[k2], ai = zi[k2];
        S.buf[f * CP + t.p] = make_float2(0.5f * (ar + br[k2]), 0.5f * (ai + bi[k2]));
        S.buf[(128 + f) * CP + t.p] = make_float2(-0.5f * (ai - bi[k2]), 0.5f * (ar - br[k2]));
    }
    __syncthreads();
    // thread t: f = 8 t + i; inclusive prefix of C over its chunk, chunk
    // totals through LDS
    float2 pc[8], d[8];
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float2 c = S.buf[(8 * t.r + i) * CP + t.p];
        acc.x += c.x;
        acc.y += c.y;
        pc[i] = acc;
        d[i] = S.buf[(128 + 8 * t.r + i) * CP + t.p];
    }
    const float2 c0 = S.buf[t.p];
    tot[t.r * CP + t.p] = acc;
    __syncthreads();
    float2 off = make_float2(-0.5f * c0.x, -0.5f * c0.y);   // S_{2f+1} = prefix(f) - C_0 / 2
    for (int u = 0; u < t.r; ++u) {
        const float2 v = tot[u * CP + t.p];
        off.x += v.x;
        off.y += v.y;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        // k = 16 t + 2 i: S_{2f} = D_f (f = 8 t + i; D_0 = 0); k + 1: S_{2f+1}
        sr[2 * i] = d[i].x;
        si[2 * i] = d[i].y;
        sr[2 * i + 1] = off.x + pc[i].x;
        si[2 * i + 1] = off.y + pc[i].y;
    }
    __syncthreads();
}

// Strided DST-I pass by the half-length algorithm (SCALE = false), or the
// last-axis pass S Lambda^{-1} S with the Parseval partials of
// (r, P^{-1} r) (SCALE = true): the scaled spectrum goes back through LDS
// in natural order and is transformed again.  Sixteen complex values per
// thread (half the registers of k_col_dst).
template <bool SCALE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
void k_col_dsth(DstArgs<float> a) {
    __shared__ Smem S;
    __shared__ float2 s_tot[16 * CP];
    __shared__ double s_red[NT / 64];
    if (a.ctrl && a.ctrl->done) return;
    const Tile t = tile_of(a.g);
    const long es = a.g.estride;
    load_tw(S, a.tw);
    // scale pass: (a_last, lc_last) at k - 1 for k = threadIdx.x (NT = 256 =
    // HN), staged in LDS between the transforms (in s_tot, free there: 40 KB
    // of LDS keeps four workgroups on a CU)
    float2 lam_k = make_float2(0.f, 0.f);
    // the line factors (P, Q below) are loaded here too, with the tile
    float fa1[2] = {0.f, 0.f}, fl1[2] = {0.f, 0.f}, fa2 = 0.f, fl2 = 0.f;
    const int o = blockIdx.x / (a.g.P1 / TX);
    if constexpr (SCALE) {
        const int k = threadIdx.x;
        if (k >= 1) lam_k = make_float2(a.a_last[k - 1], a.lc_last[k - 1]);
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int x = (int)(t.base - (long)o * a.g.ostride) + cc;
            if (x < a.g.nx) {
                fa1[cc] = a.a1[x];
                fl1[cc] = a.lc1[x];
            }
        }
        if (a.dim == 3) {
            fa2 = a.a2[o];
            fl2 = a.lc2[o];
        }
    }
    {
        // x_j = u[j - 1] for j = r + 16 m (x_0 = 0) to LDS in natural order
        float2 v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int j = t.r + 16 * m;
            v[m] = j >= 1 ? *row2(a.u, t.base + (long)(j - 1) * es) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) S.buf[(t.r + 16 * m) * CP + t.p] = v[m];
    }
    __syncthreads();
    const float c = 2.0f * a.c;   // sqrt(2 / N): the orthonormal DST-I
    float sr[16], si[16];
    dst256_from_lds(S, s_tot, t, sr, si);
    if constexpr (SCALE) {
        float P[2], Q[2];
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int x = (int)(t.base - (long)o * a.g.ostride) + cc;
            P[cc] = 0.f;
            Q[cc] = 0.f;
            if (x < a.g.nx) {
                const float a1 = fa1[cc], l1 = fl1[cc];
                if (a.dim == 2) {
                    P[cc] = a1 + l1;
                    Q[cc] = a1;
                } else {
                    P[cc] = fa2 * (a1 + l1) + fl2 * a1;
                    Q[cc] = fa2 * a1;
                }
            }
        }
        s_tot[threadIdx.x] = lam_k;
        __syncthreads();
        double acc = 0.0;
        // the scale as a compile-time choice (Lambda^{-1} or, for the
        // two-sided system, Lambda^{-1/2}): a runtime select evaluates both
        auto scale_all = [&](auto half_c) {
            constexpr bool H = decltype(half_c)::value;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k = 16 * t.r + q;
                float w0 = 0.f, w1 = 0.f;
                if (k >= 1) {
                    const float2 al = s_tot[k];
                    const float l0 = al.x * P[0] + al.y * Q[0], l1 = al.x * P[1] + al.y * Q[1];
                    const float inv0 = P[0] != 0.f ? (H ? fast_rsqrt(l0) : fast_rcp(l0)) : 0.f;
                    const float inv1 = P[1] != 0.f ? (H ? fast_rsqrt(l1) : fast_rcp(l1)) : 0.f;
                    const float s0 = c * sr[q], s1 = c * si[q];
                    w0 = s0 * inv0;
                    w1 = s1 * inv1;
                    acc += (double)s0 * (double)w0 + (double)s1 * (double)w1;
                }
                S.buf[k * CP + t.p] = make_float2(w0, w1);
            }
        };
        if (a.half) scale_all(std::true_type{});
        else scale_all(std::false_type{});
        __syncthreads();
        dst256_from_lds(S, s_tot, t, sr, si);
        if (a.partials) {
            const double sum = block_sum<NT>(acc, s_red);
            if (threadIdx.x == 0) a.partials[blockIdx.x] = sum;
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int k = 16 * t.r + q;   // DST index 1..n -> row k - 1
        if (k >= 1)
            st_nt2(a.o + t.base + (long)(k - 1) * es, t.pad0 ? 0.f : c * sr[q], t.pad1 ? 0.f : c * si[q]);
    }
}

// 32-point DFT of a line whose points 16..31 are zero (zero-padded input):
// the radix-8 DFTs over n1 (points 4 n1 + n2) have their inputs 4..7 zero.
__device__ inline void dft32_zin(float (&xr)[32], float (&xi)[32]) {
    float tr[4][8], ti[4][8];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
            tr[n2][n1] = xr[4 * n1 + n2];
            ti[n2][n1] = xi[4 * n1 + n2];
        }
#pragma unroll
        for (int n1 = 4; n1 < 8; ++n1) { tr[n2][n1] = 0.f; ti[n2][n1] = 0.f; }
        dft8_pruned<float, true, false>(tr[n2], ti[n2]);
    }
    static_for<1, 8>([&](auto K) {
        constexpr int k = decltype(K)::value;
        mul_w32<k>(tr[1][k], ti[1][k]);
        mul_w32<2 * k>(tr[2][k], ti[2][k]);
        mul_w32<3 * k>(tr[3][k], ti[3][k]);
    });
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
        const float a0r = tr[0][k1], a0i = ti[0][k1], a1r = tr[1][k1], a1i = ti[1][k1];
        const float a2r = tr[2][k1], a2i = ti[2][k1], a3r = tr[3][k1], a3i = ti[3][k1];
        const float s02r = a0r + a2r, s02i = a0i + a2i, d02r = a0r - a2r, d02i = a0i - a2i;
        const float s13r = a1r + a3r, s13i = a1i + a3i, d13r = a1r - a3r, d13i = a1i - a3i;
        xr[k1] = s02r + s13r;       xi[k1] = s02i + s13i;
        xr[k1 + 8] = d02r + d13i;   xi[k1 + 8] = d02i - d13r;
        xr[k1 + 16] = s02r - s13r;  xi[k1 + 16] = s02i - s13i;
        xr[k1 + 24] = d02r - d13i;  xi[k1 + 24] = d02i + d13r;
    }
}

// A_n along the line, (v[j-1] + 6 v[j] + v[j+1]) / 8 with zeros outside
// 0..n-1, for the rows j = r + 16 m < n a thread holds: the values go to
// LDS in natural order and the neighbours come back from there.  Ends with
// the LDS buffer free (barrier).
__device__ inline void line_stencil(Smem& S, const Tile& t, const float2 (&v)[16], float2 (&out)[16]) {
#pragma unroll
    for (int m = 0; m < 16; ++m) S.buf[(t.r + 16 * m) * CP + t.p] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int j = t.r + 16 * m;
        float2 l = make_float2(0.f, 0.f), rr = make_float2(0.f, 0.f);
        if (j > 0) l = S.buf[(j - 1) * CP + t.p];
        if (j + 1 < NN) rr = S.buf[(j + 1) * CP + t.p];
        out[m] = make_float2((l.x + 6.f * v[m].x + rr.x) * 0.125f,
                             (l.y + 6.f * v[m].y + rr.y) * 0.125f);
    }
    __syncthreads();
}

// Strided Toeplitz pass (float32, L = 512): o1 = Toep(u_fft) [+ A_n u_sten]
// with the epilogue, o2 = A_n u_fft (when set).  The Toeplitz factor is the
// circulant of length L applied as conj(FFT(conj(C) ... )): forward
// transform of the zero-padded line, Y = conj(C Z), forward transform, and
// the conjugate of the first n points.
// The epilogue (EPI_*) is a template parameter: one kernel per mode keeps
// the registers of the unused epilogues' operands out of the others.
// Register budget: two wavefronts per SIMD.  With the two line stencils the
// kernel does not fit 168 VGPRs without spilling, and the spilling build
// measured slower (106 against 76 us for the y pass at 255^3).
template <typename T, int EPI>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_col_toep(ToepArgs<T> a) {
    static_assert(std::is_same<T, float>::value, "float32 passes only");
    __shared__ Smem S;
    __shared__ float2 s_spec[L];   // read after barriers: not hoisted into registers
    __shared__ double s_red[NT / 64];
    if (a.ctrl && a.ctrl->done) return;
    const Tile t = tile_of(a.g);
    const long es = a.g.estride;
    const int o = blockIdx.x / (a.g.P1 / TX);
    const int x = (int)(t.base - (long)o * a.g.ostride);
    load_tw(S, a.tw);
    stage_table(s_spec, a.spec);
    float xr[32], xi[32];
    {
        float2 v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int j = t.r + 16 * m;
            v[m] = j < NN ? *row2(a.u_fft, t.base + (long)j * es) : make_float2(0.f, 0.f);
        }
        if (a.o2) {
            float2 st[16];
            line_stencil(S, t, v, st);
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int j = t.r + 16 * m;
                if (j < NN)
                    st_nt2(a.o2 + t.base + (long)j * es, t.pad0 ? 0.f : st[m].x,
                           t.pad1 ? 0.f : st[m].y);
            }
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            xr[m] = v[m].x;
            xi[m] = v[m].y;
        }
    }
    dft32_zin(xr, xi);
    float yr2[2][16], yi2[2][16];
    transpose_fwd_half(S, t, 0, xr, xi, yr2[0], yi2[0]);
    transpose_fwd_half(S, t, 1, xr, xi, yr2[1], yi2[1]);
    // the stencil operand's rows are loaded here, in flight during the
    // spectral products and the inverse transposes (the offset is made
    // opaque so that the loads are not hoisted to the top of the kernel,
    // where their registers would stay live through both transforms)
    float2 vs[16];
    if (a.u_sten) {
        long off = t.base;
        asm volatile("" : "+v"(off));
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int j = t.r + 16 * m;
            vs[m] = j < NN ? *row2(a.u_sten, off + (long)j * es) : make_float2(0.f, 0.f);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k1 = t.r + 16 * h;
        float (&yr)[16] = yr2[h];
        float (&yi)[16] = yi2[h];
        dft16<16>(yr, yi);
        // Y = conj(C Z) at f = k1 + 32 k2
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            const int f = k1 + 32 * k2;
            const float2 c = s_spec[f];
            const float zr = yr[k2], zi = yi[k2];
            yr[k2] = c.x * zr - c.y * zi;
            yi[k2] = -(c.x * zi + c.y * zr);
        }
        dft16<16>(yr, yi);
        transpose_inv_half(S, t, h, yr, yi, xr, xi);
    }
    dft32<16>(xr, xi);
    // rows j = r + 16 j2 < n: out = conj(Y) [+ A_n u_sten] and the epilogue
    float2 sten[16];
    if (a.u_sten) {
        line_stencil(S, t, vs, sten);
    } else {
#pragma unroll
        for (int m = 0; m < 16; ++m) sten[m] = make_float2(0.f, 0.f);
    }
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int j = t.r + 16 * m;
        if (j >= NN) continue;
        const long gi = t.base + (long)j * es;
        float v0 = xr[m] + sten[m].x, v1 = -xi[m] + sten[m].y;
        if (t.pad0) v0 = 0.f;
        if (t.pad1) v1 = 0.f;
        if constexpr (EPI == EPI_ADD_F) {
            const long fo = (long)a.g.n1 * ((long)j * a.g.fr_i + (long)o * a.g.fr_o);
            if (x < a.g.n1) v0 += (float)(a.dt * a.F[x + fo]);
            if (x + 1 < a.g.n1) v1 += (float)(a.dt * a.F[x + 1 + fo]);
        } else if constexpr (EPI == EPI_DOT_P) {
            const float2 d = *row2(a.dot_p, gi);
            acc += (double)d.x * (double)v0 + (double)d.y * (double)v1;
        } else if constexpr (EPI == EPI_RESID) {
            const float2 b = *row2(a.b, gi);
            v0 = b.x - v0;
            v1 = b.y - v1;
            acc += (double)v0 * (double)v0 + (double)v1 * (double)v1;
        }
        st_nt2(a.o1 + gi, v0, v1);
    }
    if constexpr (EPI == EPI_DOT_P || EPI == EPI_RESID) {
        const double s = block_sum<NT>(acc, s_red);
        if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
    }
}

}  // namespace colx
}  // namespace fsd
