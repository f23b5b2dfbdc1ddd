// DST-I of the float32 preconditioner as dense products on the matrix cores.
//
// For an axis with n <= 256 the orthonormal DST-I matrix S (n x n,
// S[k][j] = sqrt(2/(n+1)) sin(pi (j+1)(k+1)/(n+1)), Section 3) is applied as
// a bf16 MFMA product with float32 accumulation.  S is rounded to bf16 once
// (a fixed, symmetric, nonsingular matrix, so S Lambda^{-1} S stays a
// symmetric positive definite preconditioner); each float32 input value is
// split into bf16 hi + lo, so the input is carried to 16 significant bits
// and the map stays linear to that accuracy.  The products cost 2 x 2n
// flop per value and axis, far below the MFMA rate.  Measured at 255^3 these
// passes (58 / 79 / 206 us for x / y / fused last axis) do not beat the FFT
// passes (53 / 58 / 124 us): they are latency bound at one or two
// wavefronts per SIMD, so the FFT path is the default (dst_mfma = 0).
//
// S is stored as MFMA fragments F[s][t] (s: 16-wide K step, t: 16-row
// tile, 64 lanes x 4 bf16): lane l holds S[16 t + l % 16][16 s + 4 (l / 16) + e].
// Because S is symmetric the same fragment is the A operand (rows of S) of
// a column pass and the B operand (columns of S^T = S) of a row pass.  A
// workgroup stages the NT fragments of one K step in LDS (NT x 512 bytes,
// contiguous) and its four wavefronts share them.
#include "fsd_internal.h"

namespace fsd {

namespace {

typedef short g_s4 __attribute__((ext_vector_type(4)));
typedef short g_s8 __attribute__((ext_vector_type(8)));
typedef __bf16 g_bf8 __attribute__((ext_vector_type(8)));
typedef float g_f4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 32 bf16 product (gfx950) over 16 K values carried twice:
// the A operand's halves a0 | a1 and the B operand's halves b0 | b1 fill the
// instruction's 32 K slots in the same order, so D += a0 b0 + a1 b1 with
// each pair taken over the same 16 K values (the hardware pairs A and B K
// slots by lane and element alike, whatever order it sums them in).
__device__ inline g_f4 g_mfma_pair(const g_s4& a0, const g_s4& a1, const g_s4& b0, const g_s4& b1,
                                   const g_f4& c) {
    const g_s8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const g_s8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(g_bf8, a),
                                                   __builtin_bit_cast(g_bf8, b), c, 0, 0, 0);
}

__device__ inline unsigned short g_f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(u >> 16);
}
__device__ inline float g_bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// v = hi + lo with hi = bf16(v), lo = bf16(v - hi).
__device__ inline void g_split(const float (&v)[4], g_s4& hi, g_s4& lo) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const unsigned short h = g_f2bf(v[e]);
        hi[e] = (short)h;
        lo[e] = (short)g_f2bf(v[e] - g_bf2f(h));
    }
}

__device__ inline double g_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Copy the NT fragments of K step s into LDS (all threads of the block).
template <int NT>
__device__ inline void g_stage(const void* frag, int s, g_s4* lds) {
    const g_s4* src = reinterpret_cast<const g_s4*>(frag) + (long)s * NT * 64;
    for (int i = threadIdx.x; i < NT * 64; i += 256) lds[i] = src[i];
}

// ------------------------------------------------------------ x axis
// One wavefront: MR = 2 16-row tiles x all n16 outputs, so that each S
// fragment read from LDS feeds two products (one row tile per wavefront
// runs at higher occupancy but measured slower at n = 255: 71 against
// 58 us).  Input rows have pitch P1 >= n16 and zero padding, so the K range
// needs no guard.
template <int NT>
constexpr int gdst_row_tiles() { return 2; }

template <int NT>
__global__ __launch_bounds__(256) void k_gdst_row(GdstArgs a) {
    constexpr int MR = gdst_row_tiles<NT>();
    __shared__ g_s4 fs[2][NT * 64];
    if (a.ctrl && a.ctrl->done) return;
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long r0 = wave * 16 * MR;
    const long nrows = a.g.nrows;
    const int P1 = a.g.P1, n = a.g.n;
    const int c = lane & 15, g = lane >> 4;
    g_f4 acc[MR][NT];
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = g_f4{0.f, 0.f, 0.f, 0.f};
    g_stage<NT>(a.frag, 0, fs[0]);
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        g_s4 hi[MR], lo[MR];
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const long row = r0 + m * 16 + c;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (row < nrows) {
                const float4 w = *reinterpret_cast<const float4*>(a.u + row * P1 + s * 16 + 4 * g);
                v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
            }
            g_split(v, hi[m], lo[m]);
        }
        __syncthreads();                                   // fragments of step s ready
        if (s + 1 < NT) g_stage<NT>(a.frag, s + 1, fs[(s + 1) & 1]);
        const g_s4* F = fs[s & 1] + lane;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const g_s4 b = F[t * 64];
#pragma unroll
            for (int m = 0; m < MR; ++m) acc[m][t] = g_mfma_pair(hi[m], lo[m], b, b, acc[m][t]);
        }
    }
    if (r0 >= nrows) return;
    // D[row][k]: lane holds k = 16 t + c for rows 16 m + 4 g + r
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = r0 + m * 16 + 4 * g + r;
            if (row >= nrows) continue;
            float* o = a.o + row * P1;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int k = 16 * t + c;
                o[k] = k < n ? acc[m][t][r] : 0.f;
            }
            for (int k = 16 * NT + c; k < P1; k += 16) o[k] = 0.f;
        }
}

// ------------------------------------------------------------ y / z axes
// One wavefront: 16 consecutive x columns of one outer index, all n16
// outputs along the line.  Columns x >= nx hold zeros and produce zeros.
template <int NT, bool SCALE>
__global__ __launch_bounds__(256) void k_gdst_col(GdstArgs a) {
    __shared__ g_s4 fs[2][NT * 64];
    __shared__ double s_red[4];
    if (a.ctrl && a.ctrl->done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long wave = (long)blockIdx.x * 4 + wv;
    const int P1 = a.g.P1, n = a.g.n;
    const int nxt = P1 / 16;
    const long nw = (long)nxt * a.g.n_outer;
    const bool live = wave < nw;
    const int c = lane & 15, g = lane >> 4;
    const int xt = live ? (int)(wave % nxt) : 0;
    const int o = live ? (int)(wave / nxt) : 0;
    const int x = xt * 16 + c;
    const long es = a.g.estride;
    const long base = (long)o * a.g.ostride + x;
    double part = 0.0;
    g_f4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = g_f4{0.f, 0.f, 0.f, 0.f};
    g_stage<NT>(a.frag, 0, fs[0]);
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 16 * s + 4 * g + e;
            v[e] = (live && j < n) ? a.u[base + (long)j * es] : 0.f;
        }
        g_s4 hi, lo;
        g_split(v, hi, lo);
        __syncthreads();
        if (s + 1 < NT) g_stage<NT>(a.frag, s + 1, fs[(s + 1) & 1]);
        const g_s4* F = fs[s & 1] + lane;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const g_s4 f = F[t * 64];
            acc[t] = g_mfma_pair(f, f, hi, lo, acc[t]);
        }
    }
    if constexpr (SCALE) {
        // Lambda[k, o, x] = a_last[k] P + lc_last[k] Q (Section 3), zero on
        // padding columns; Parseval: (r, P^{-1} r) = sum (S r)^2 / Lambda.
        float Pv = 0.f, Qv = 0.f;
        if (live && x < a.g.nx) {
            const float a1 = a.a1[x], l1 = a.lc1[x];
            if (a.dim == 2) {
                Pv = a1 + l1;
                Qv = a1;
            } else {
                const float a2 = a.a2[o], l2 = a.lc2[o];
                Pv = a2 * (a1 + l1) + l2 * a1;
                Qv = a2 * a1;
            }
        }
        // the scaled values are the B operands (K = k) of the inverse
        // transform: D's lane layout (k = 16 t + 4 g + r) is the B layout
        // of K step t
        g_f4 acc2[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc2[t] = g_f4{0.f, 0.f, 0.f, 0.f};
        __syncthreads();
        g_stage<NT>(a.frag, 0, fs[0]);
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            float w[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * s + 4 * g + r;
                float wk = 0.f;
                if (k < n && Pv != 0.f) {
                    const float sv = acc[s][r];
                    const float lam = a.a_last[k] * Pv + a.lc_last[k] * Qv;
                    wk = a.half ? sv * __builtin_amdgcn_rsqf(lam) : sv / lam;
                    part += (double)sv * (double)wk;
                }
                w[r] = wk;
            }
            g_s4 hi, lo;
            g_split(w, hi, lo);
            __syncthreads();
            if (s + 1 < NT) g_stage<NT>(a.frag, s + 1, fs[(s + 1) & 1]);
            const g_s4* F = fs[s & 1] + lane;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const g_s4 f = F[t * 64];
                acc2[t] = g_mfma_pair(f, f, hi, lo, acc2[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = acc2[t];
    }
    if (live) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * t + 4 * g + r;
                if (k < n) a.o[base + (long)k * es] = acc[t][r];
            }
    }
    if constexpr (SCALE) {
        if (a.partials) {
            const double sw = g_wave_sum(part);
            if (lane == 0) s_red[wv] = sw;
            __syncthreads();
            if (threadIdx.x == 0) a.partials[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
        }
    }
}

template <bool SCALE>
hipError_t col_dispatch(int nt, const GdstArgs& a, int g, hipStream_t s) {
    switch (nt) {
#define GDST_C(NT_) case NT_: hipLaunchKernelGGL((k_gdst_col<NT_, SCALE>), dim3(g), dim3(256), 0, s, a); break;
        GDST_C(1) GDST_C(2) GDST_C(3) GDST_C(4) GDST_C(6) GDST_C(8) GDST_C(12) GDST_C(16)
#undef GDST_C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool gdst_supported(int n) {
    const int nt = (n + 15) / 16;
    return n >= 1 && (nt == 1 || nt == 2 || nt == 3 || nt == 4 || nt == 6 || nt == 8 || nt == 12 ||
                      nt == 16);
}

hipError_t launch_gdst_row(const GdstArgs& a, hipStream_t s) {
    const int nt = (a.g.n + 15) / 16;
    switch (nt) {
#define GDST_R(NT_)                                                                         \
    case NT_: {                                                                             \
        constexpr long rows = 16L * gdst_row_tiles<NT_>();                                   \
        const int g = (int)(((a.g.nrows + rows - 1) / rows + 3) / 4);                       \
        if (g) hipLaunchKernelGGL((k_gdst_row<NT_>), dim3(g), dim3(256), 0, s, a);          \
        break;                                                                              \
    }
        GDST_R(1) GDST_R(2) GDST_R(3) GDST_R(4) GDST_R(6) GDST_R(8) GDST_R(12) GDST_R(16)
#undef GDST_R
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int gdst_col_blocks(const PassGeo& g) { return (int)(((long)(g.P1 / 16) * g.n_outer + 3) / 4); }

hipError_t launch_gdst_col(const GdstArgs& a, bool scale, int* nblocks, hipStream_t s) {
    const int nt = (a.g.n + 15) / 16;
    const int g = gdst_col_blocks(a.g);
    if (nblocks) *nblocks = g;
    if (g == 0) return hipSuccess;
    return scale ? col_dispatch<true>(nt, a, g, s) : col_dispatch<false>(nt, a, g, s);
}

}  // namespace fsd
