// Kernels of the warm-start network: MFMA implicit-GEMM 3x3x3 convolution
// (forward, input gradient through transposed weights, weight gradient),
// pooling and upsampling with their adjoints, features, loss and Adam.
#include "fsd_nn.h"

namespace fsd {

namespace {

typedef float nn_f4 __attribute__((ext_vector_type(4)));
typedef short nn_s8 __attribute__((ext_vector_type(8)));
typedef __bf16 nn_bf8 __attribute__((ext_vector_type(8)));

// Two consecutive 16-value K steps in one 16 x 16 x 32 bf16 product (gfx950):
// A = a0 | a1 and B = b0 | b1 fill the instruction's 32 K slots in the same
// order, so D += a0 b0 + a1 b1 (the hardware pairs A and B K slots by lane
// and element alike, whatever order it sums them in).
__device__ inline nn_f4 mfma_k32(const nn_s4& a0, const nn_s4& a1, const nn_s4& b0, const nn_s4& b1,
                                 const nn_f4& c) {
    const nn_s8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const nn_s8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(nn_bf8, a),
                                                   __builtin_bit_cast(nn_bf8, b), c, 0, 0, 0);
}

__device__ inline bf16_t f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)            // inf / nan: keep, quiet the nan
        return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);                  // round to nearest even
    return (bf16_t)(u >> 16);
}
__device__ inline float bf2f(bf16_t h) { return __uint_as_float(((unsigned)h) << 16); }
__device__ inline bool bf_pos(bf16_t h) { return (h & 0x8000u) == 0 && (h & 0x7fffu) != 0; }

struct U4 {
    bf16_t v[4];
};
__device__ inline U4 ld4(const bf16_t* p) {
    const uint2 w = *reinterpret_cast<const uint2*>(p);
    U4 r;
    r.v[0] = (bf16_t)(w.x & 0xffffu); r.v[1] = (bf16_t)(w.x >> 16);
    r.v[2] = (bf16_t)(w.y & 0xffffu); r.v[3] = (bf16_t)(w.y >> 16);
    return r;
}
__device__ inline void st4(bf16_t* p, const float (&f)[4]) {
    uint2 w;
    w.x = (unsigned)f2bf(f[0]) | ((unsigned)f2bf(f[1]) << 16);
    w.y = (unsigned)f2bf(f[2]) | ((unsigned)f2bf(f[3]) << 16);
    *reinterpret_cast<uint2*>(p) = w;
}

__device__ inline double nn_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
// Workgroup sum of 256 threads, valid in thread 0.
__device__ inline double nn_block_sum(double v, double* sb) {
    v = nn_wave_sum(v);
    if ((threadIdx.x & 63) == 0) sb[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (sb[0] + sb[1]) + (sb[2] + sb[3]);
    return s;
}

// ---------------------------------------------------------------- weights

__global__ void k_nn_frag(const float* __restrict__ W, int cin, int cout, int transposed,
                          nn_s4* __restrict__ frag, int ks, int mb, int kcin_p) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)ks * mb * 64;
    if (i >= total) return;
    const int lane = (int)(i % 64);
    const int mbi = (int)((i / 64) % mb);
    const int s = (int)(i / (64L * mb));
    const int row = mbi * 16 + (lane & 15);
    nn_s4 out;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int k = 16 * s + 4 * (lane >> 4) + e;
        const int tap = k / kcin_p, col = k - tap * kcin_p;
        float v = 0.f;
        if (tap < 27) {
            if (!transposed) {
                if (row < cout && col < cin) v = W[((long)row * cin + col) * 27 + tap];
            } else {
                if (row < cin && col < cout) v = W[((long)col * cin + row) * 27 + (26 - tap)];
            }
        }
        out[e] = (short)f2bf(v);
    }
    frag[i] = out;
}

// ---------------------------------------------------------------- conv

// Workgroup tile: 16 x positions x 4 y rows x R z planes of output voxels,
// all output channels (MB blocks of 16).  The input block with a one-voxel
// halo, 18 x 6 x (R + 2) voxels of CP channels, is staged once in LDS
// (voxel pitch CP + 4 halfwords against bank conflicts); wavefront w
// computes the row y0 + w of the R planes.  Per K-step (16 values of
// K = (tap, channel)) each lane reads its 4 channels of one tap from LDS
// and the MB A fragments from global memory (shared by the R rows).
// With a.up set, the staged input is in[v] + up[v / 2] (the decoder's
// upsample-and-add, rounded to bf16 as the separate kernel does).
constexpr int kConvTY = 4;

// LDS offset (halfwords) of tap t = 9 dz + 3 dy + dx in the staged block.
template <int TYH, int TX, int P>
__device__ constexpr int tap_off(int t) {
    return (((t / 9) * TYH + (t / 3) % 3) * TX + t % 3) * P;
}

template <int CP, int MB, int R, bool K32>
__global__ __launch_bounds__(256) void k_nn_conv(NnConvArgs a) {
    extern __shared__ bf16_t tile[];
    constexpr int P = CP + 4, Q4 = CP / 4, TX = 18, TYH = kConvTY + 2, TZH = R + 2;
    constexpr int KS = (27 * CP + 15) / 16;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nxb = (a.d.W + 15) >> 4, nyb = (a.d.H + kConvTY - 1) / kConvTY;
    const int nzb = (a.d.D + R - 1) / R;
    long bid = blockIdx.x;
    const int xb = (int)(bid % nxb);
    bid /= nxb;
    const int yb = (int)(bid % nyb);
    bid /= nyb;
    const int zb = (int)(bid % nzb);
    const int b = (int)(bid / nzb);
    const int x0 = xb * 16, y0 = yb * kConvTY, z0 = zb * R;
    const long plane = (long)a.d.H * a.d.W;
    const bf16_t* inb = a.in + (long)b * a.d.D * plane * CP;
    const long uplane = (long)a.upd.H * a.upd.W;
    const bf16_t* upb = a.up ? a.up + (long)b * a.upd.D * uplane * CP : nullptr;
    // stage the input block: 8-byte words, zero outside the grid.  All loads
    // of a thread are issued before the first LDS store (the loop is
    // unrolled), so the block costs one memory latency, not one per word.
    constexpr int NWORDS = TX * TYH * TZH * Q4;
    constexpr int NIT = (NWORDS + 255) / 256;
    uint2 val[NIT], upv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = threadIdx.x + it * 256;
        const int q = i % Q4;
        const int vx = (i / Q4) % TX;
        const int vy = (i / (Q4 * TX)) % TYH;
        const int vz = i / (Q4 * TX * TYH);
        const int zz = z0 + vz - 1, yy = y0 + vy - 1, xx = x0 + vx - 1;
        val[it] = make_uint2(0u, 0u);
        upv[it] = make_uint2(0u, 0u);
        if (i < NWORDS && zz >= 0 && zz < a.d.D && yy >= 0 && yy < a.d.H && xx >= 0 &&
            xx < a.d.W) {
            val[it] = *reinterpret_cast<const uint2*>(
                inb + ((long)zz * plane + (long)yy * a.d.W + xx) * CP + 4 * q);
            if (upb)
                upv[it] = *reinterpret_cast<const uint2*>(
                    upb + ((long)(zz >> 1) * uplane + (long)(yy >> 1) * a.upd.W + (xx >> 1)) * CP +
                    4 * q);
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = threadIdx.x + it * 256;
        if (i < NWORDS) {
            const int q = i % Q4;
            const int vx = (i / Q4) % TX;
            const int vy = (i / (Q4 * TX)) % TYH;
            const int vz = i / (Q4 * TX * TYH);
            uint2 v = val[it];
            if (upb) {
                const U4 k = ld4(reinterpret_cast<const bf16_t*>(&val[it]));
                const U4 c = ld4(reinterpret_cast<const bf16_t*>(&upv[it]));
                float f[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) f[e] = bf2f(c.v[e]) + bf2f(k.v[e]);
                st4(reinterpret_cast<bf16_t*>(&v), f);
            }
            *reinterpret_cast<uint2*>(tile + ((vz * TYH + vy) * TX + vx) * P + 4 * q) = v;
        }
    }
    __syncthreads();
    const int n = lane & 15, g = lane >> 4;
    nn_f4 acc[R][MB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < MB; ++m) acc[r][m] = nn_f4{0.f, 0.f, 0.f, 0.f};
    // K index k = 16 s + 4 g + e = tap * CP + channel.  The loop over the KS
    // K-steps is fully unrolled, so the tap of each step (and its LDS
    // offset) is a constant: for CP >= 16 one tap per step and the lane
    // group only picks the channels; for CP = 8 (4) a step spans 2 (4)
    // taps, selected by the lane group.
    const nn_s4* fr = a.frag + lane;
    const bf16_t* tw = tile + (w * TX + n) * P + (CP >= 16 ? 4 * g : CP == 8 ? 4 * (g & 1) : 0);
    // LDS offset of this lane's 4 channels at K step s, and whether its tap
    // exists (the last step may run past tap 26)
    auto step_off = [&](int s, bool& tv) -> int {
        tv = true;
        if constexpr (CP >= 16) {
            return tap_off<TYH, TX, P>((16 * s) / CP) + (16 * s) % CP;
        } else if constexpr (CP == 8) {
            const int t0 = 2 * s, t1 = 2 * s + 1;
            if (t1 >= 27) tv = (g >> 1) == 0;
            return (g >> 1) ? tap_off<TYH, TX, P>(t1) : tap_off<TYH, TX, P>(t0);
        } else {
            const int t = 4 * s;
            if (t + 3 >= 27) tv = t + g < 27;
            return g == 0 ? tap_off<TYH, TX, P>(t) : g == 1 ? tap_off<TYH, TX, P>(t + 1)
                 : g == 2 ? tap_off<TYH, TX, P>(t + 2) : tap_off<TYH, TX, P>(t + 3);
        }
    };
    // K32: K steps in pairs (s0 = 2 q, s1 = 2 q + 1), one K = 32 product per
    // pair (an odd last step pairs with zeros); else one K = 16 product per
    // step
    if constexpr (!K32) {
#pragma unroll
        for (int s0 = 0; s0 < KS; ++s0) {
            nn_s4 av[MB];
#pragma unroll
            for (int m = 0; m < MB; ++m) av[m] = fr[(s0 * MB + m) * 64];
            bool tv0;
            const int off0 = step_off(s0, tv0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                nn_s4 bv = {0, 0, 0, 0};
                if (tv0) bv = *reinterpret_cast<const nn_s4*>(tw + off0 + r * (TYH * TX * P));
#pragma unroll
                for (int m = 0; m < MB; ++m)
                    acc[r][m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[m], bv, acc[r][m], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int s0 = 0; K32 && s0 < KS; s0 += 2) {
        const int s1 = s0 + 1;
        const bool has1 = s1 < KS;
        nn_s4 av0[MB], av1[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            av0[m] = fr[(s0 * MB + m) * 64];
            av1[m] = has1 ? fr[(s1 * MB + m) * 64] : nn_s4{0, 0, 0, 0};
        }
        bool tv0, tv1 = false;
        const int off0 = step_off(s0, tv0);
        const int off1 = has1 ? step_off(s1, tv1) : 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            nn_s4 bv0 = {0, 0, 0, 0}, bv1 = {0, 0, 0, 0};
            if (tv0) bv0 = *reinterpret_cast<const nn_s4*>(tw + off0 + r * (TYH * TX * P));
            if (has1 && tv1) bv1 = *reinterpret_cast<const nn_s4*>(tw + off1 + r * (TYH * TX * P));
#pragma unroll
            for (int m = 0; m < MB; ++m) acc[r][m] = mfma_k32(av0[m], av1[m], bv0, bv1, acc[r][m]);
        }
    }
    const int x = x0 + n, y = y0 + w;
    if (x >= a.d.W || y >= a.d.H) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int z = z0 + r;
        if (z >= a.d.D) break;
        const long vox = (((long)b * a.d.D + z) * a.d.H + y) * a.d.W + x;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int co0 = m * 16 + 4 * g;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = co0 + e;
                float t = acc[r][m][e];
                if (co < a.cout) {
                    if (a.bias) t += a.bias[co];
                    if (a.relu) t = fmaxf(t, 0.f);
                } else {
                    t = 0.f;
                }
                v[e] = t;
            }
            if (a.out && co0 < a.cout_p) st4(a.out + vox * a.cout_p + co0, v);
            if (a.out32 && co0 == 0) a.out32[vox] = v[0];
        }
    }
}

// ---------------------------------------------------------------- pool / up

__device__ inline void unvox(long v, const NnDims& d, int& b, int& z, int& y, int& x) {
    x = (int)(v % d.W);
    v /= d.W;
    y = (int)(v % d.H);
    v /= d.H;
    z = (int)(v % d.D);
    b = (int)(v / d.D);
}
__device__ inline long vox_of(const NnDims& d, int b, int z, int y, int x) {
    return (((long)b * d.D + z) * d.H + y) * d.W + x;
}

__global__ void k_nn_pool(const bf16_t* __restrict__ in, bf16_t* __restrict__ out, NnDims f,
                          NnDims c, int cp) {
    const int q4 = cp >> 2;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.vox() * q4) return;
    const int q = (int)(i % q4);
    int b, z, y, x;
    unvox(i / q4, c, b, z, y, x);
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int zz = 2 * z + dz, yy = 2 * y + dy, xx = 2 * x + dx;
                if (zz < f.D && yy < f.H && xx < f.W) {
                    const U4 w = ld4(in + vox_of(f, b, zz, yy, xx) * cp + 4 * q);
#pragma unroll
                    for (int e = 0; e < 4; ++e) s[e] += bf2f(w.v[e]);
                }
            }
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] *= 0.125f;
    st4(out + (i / q4) * cp + 4 * q, s);
}

__global__ void k_nn_upadd(const bf16_t* __restrict__ coarse, const bf16_t* __restrict__ skip,
                           bf16_t* __restrict__ out, NnDims f, NnDims c, int cp) {
    const int q4 = cp >> 2;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.vox() * q4) return;
    const int q = (int)(i % q4);
    int b, z, y, x;
    unvox(i / q4, f, b, z, y, x);
    const U4 a = ld4(coarse + vox_of(c, b, z >> 1, y >> 1, x >> 1) * cp + 4 * q);
    const U4 k = ld4(skip + (i / q4) * cp + 4 * q);
    float s[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] = bf2f(a.v[e]) + bf2f(k.v[e]);
    st4(out + (i / q4) * cp + 4 * q, s);
}

__global__ void k_nn_up_bwd_mask(const bf16_t* __restrict__ gf, const bf16_t* __restrict__ act,
                                 bf16_t* __restrict__ gc, NnDims f, NnDims c, int cp) {
    const int q4 = cp >> 2;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.vox() * q4) return;
    const int q = (int)(i % q4);
    int b, z, y, x;
    unvox(i / q4, c, b, z, y, x);
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int zz = 2 * z + dz, yy = 2 * y + dy, xx = 2 * x + dx;
                if (zz < f.D && yy < f.H && xx < f.W) {
                    const U4 w = ld4(gf + vox_of(f, b, zz, yy, xx) * cp + 4 * q);
#pragma unroll
                    for (int e = 0; e < 4; ++e) s[e] += bf2f(w.v[e]);
                }
            }
    const U4 m = ld4(act + (i / q4) * cp + 4 * q);
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] = bf_pos(m.v[e]) ? s[e] : 0.f;
    st4(gc + (i / q4) * cp + 4 * q, s);
}

__global__ void k_nn_pool_bwd_add_mask(const bf16_t* __restrict__ gc, const bf16_t* __restrict__ gs,
                                       const bf16_t* __restrict__ act, bf16_t* __restrict__ g,
                                       NnDims f, NnDims c, int cp) {
    const int q4 = cp >> 2;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.vox() * q4) return;
    const int q = (int)(i % q4);
    int b, z, y, x;
    unvox(i / q4, f, b, z, y, x);
    const U4 a = ld4(gc + vox_of(c, b, z >> 1, y >> 1, x >> 1) * cp + 4 * q);
    const U4 k = ld4(gs + (i / q4) * cp + 4 * q);
    const U4 m = ld4(act + (i / q4) * cp + 4 * q);
    float s[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        s[e] = bf_pos(m.v[e]) ? bf2f(k.v[e]) + 0.125f * bf2f(a.v[e]) : 0.f;
    st4(g + (i / q4) * cp + 4 * q, s);
}

// ---------------------------------------------------------------- wgrad

// One wavefront: a 16 (output channels) x 16 (K columns) tile of dW over one
// chunk of voxels; each MFMA takes 32 voxels (two groups of 16, 4 per lane
// group each).
__global__ __launch_bounds__(256) void k_nn_wgrad(NnWgradArgs a, int mbn, int kn, long nwaves) {
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int nb = (int)(wave % kn);
    const int mb = (int)((wave / kn) % mbn);
    const long chunk = wave / ((long)kn * mbn);
    const int j = lane & 15, g = lane >> 4;
    const int co = mb * 16 + j;                       // A row of this lane
    const int kk = nb * 16 + j;                       // B column of this lane
    const int tap = kk >> a.cin_shift, ci = kk & (a.cin_p - 1);
    const bool kval = tap < 27;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const long V = a.d.vox();
    const long v0 = chunk * a.vchunk;
    const long v1 = v0 + a.vchunk < V ? v0 + a.vchunk : V;
    nn_f4 acc = {0.f, 0.f, 0.f, 0.f};
    // 16 voxels (4 per lane group) of the K range
    auto load = [&](long vb, nn_s4& av, nn_s4& bv) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const long v = vb + 4 * g + e;
            short ga = 0, xb = 0;
            if (v < v1) {
                if (co < a.cout) ga = (short)a.gout[v * a.cout_p + co];
                if (kval) {
                    int b, z, y, x;
                    unvox(v, a.d, b, z, y, x);
                    const int zz = z + dz, yy = y + dy, xx = x + dx;
                    if (zz >= 0 && zz < a.d.D && yy >= 0 && yy < a.d.H && xx >= 0 && xx < a.d.W)
                        xb = (short)a.in[vox_of(a.d, b, zz, yy, xx) * a.cin_p + ci];
                }
            }
            av[e] = ga;
            bv[e] = xb;
        }
    };
    // 32 voxels per K = 32 product (voxels past v1 load as zeros)
    for (long vb = v0; vb < v1; vb += 32) {
        nn_s4 av0, bv0, av1, bv1;
        load(vb, av0, bv0);
        load(vb + 16, av1, bv1);
        acc = mfma_k32(av0, av1, bv0, bv1, acc);
    }
    // D[row = output channel][col = K column]: lane holds col j, rows 4g + r
    const long pitch = (long)kn * 16;
    float* p = a.partials + chunk * (long)mbn * 16 * pitch;
#pragma unroll
    for (int r = 0; r < 4; ++r) p[(long)(mb * 16 + 4 * g + r) * pitch + kk] = acc[r];
}

// Bias partials: one thread per (chunk, channel).
__global__ void k_nn_bgrad(NnWgradArgs a, long nchunks) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nchunks * a.cout) return;
    const int co = (int)(i % a.cout);
    const long chunk = i / a.cout;
    const long V = a.d.vox();
    const long v0 = chunk * a.vchunk;
    const long v1 = v0 + a.vchunk < V ? v0 + a.vchunk : V;
    float s = 0.f;
    for (long v = v0; v < v1; ++v) s += bf2f(a.gout[v * a.cout_p + co]);
    a.bpartials[i] = s;
}

// Fixed-order reduction of the chunk partials into gW[o][i][tap] and gb[o].
__global__ void k_nn_wgrad_reduce(NnWgradArgs a, int mbn, int kn, long nchunks) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nw = (long)a.cout * a.cin * 27;
    if (i < nw) {
        const int tap = (int)(i % 27);
        const int ci = (int)((i / 27) % a.cin);
        const int co = (int)(i / (27L * a.cin));
        const long pitch = (long)kn * 16;
        const long cstride = (long)mbn * 16 * pitch;
        const long off = (long)co * pitch + (long)tap * a.cin_p + ci;
        float s = 0.f;
        for (long c = 0; c < nchunks; ++c) s += a.partials[c * cstride + off];
        a.gW[i] = s;
    } else if (i < nw + a.cout) {
        const int co = (int)(i - nw);
        float s = 0.f;
        for (long c = 0; c < nchunks; ++c) s += a.bpartials[c * a.cout + co];
        a.gb[co] = s;
    }
}

// ---------------------------------------------------------------- features

// du = u - uprev and df = dt (F - Fprev) at element e (absent arrays: zero).
__device__ inline void nn_incr(const double* u, const double* up, const double* F,
                               const double* Fp, double dt, long e, double& du, double& df) {
    du = up ? u[e] - up[e] : 0.0;
    df = dt * ((F ? F[e] : 0.0) - (Fp ? Fp[e] : 0.0));
}

__global__ __launch_bounds__(256) void k_nn_sumsq(const double* __restrict__ u,
                                                  const double* __restrict__ up,
                                                  const double* __restrict__ F,
                                                  const double* __restrict__ Fp, double dt, long N,
                                                  double* __restrict__ partials) {
    __shared__ double sb[4];
    double su = 0.0, sf = 0.0;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < N; e += (long)gridDim.x * 256) {
        double du, df;
        nn_incr(u, up, F, Fp, dt, e, du, df);
        su += du * du;
        sf += df * df;
    }
    const double S1 = nn_block_sum(su, sb);
    __syncthreads();
    const double S2 = nn_block_sum(sf, sb);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = S1;
        partials[gridDim.x + blockIdx.x] = S2;
    }
}

__global__ __launch_bounds__(256) void k_nn_scale_fin(const double* __restrict__ partials, int np,
                                                      long N, double* s_out) {
    __shared__ double sb[4];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) {
        a += partials[i];
        b += partials[np + i];
    }
    const double S1 = nn_block_sum(a, sb);
    __syncthreads();
    const double S2 = nn_block_sum(b, sb);
    if (threadIdx.x == 0) *s_out = sqrt(S1 / (double)N) + sqrt(S2 / (double)N) + 1e-30;
}

__global__ void k_nn_feat_bf16(const double* __restrict__ u, const double* __restrict__ up,
                               const double* __restrict__ F, const double* __restrict__ Fp, double dt,
                               const double* __restrict__ s, float l0, float l1, float l2, long N,
                               bf16_t* __restrict__ x) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const double inv = 1.0 / *s;
    double du, df;
    nn_incr(u, up, F, Fp, dt, e, du, df);
    const float v0[4] = {(float)(du * inv), (float)(df * inv), l0, l1};
    const float v1[4] = {l2, 0.f, 0.f, 0.f};
    st4(x + e * 8, v0);
    st4(x + e * 8 + 4, v1);
}

__global__ void k_nn_feat_f32(const double* __restrict__ u, const double* __restrict__ up,
                              const double* __restrict__ F, const double* __restrict__ Fp,
                              const double* __restrict__ un, double dt, const double* __restrict__ s,
                              float l0, float l1, float l2, long N, float* __restrict__ x,
                              float* __restrict__ t) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const double inv = 1.0 / *s;
    double du, df;
    nn_incr(u, up, F, Fp, dt, e, du, df);
    x[e] = (float)(du * inv);
    x[N + e] = (float)(df * inv);
    x[2 * N + e] = l0;
    x[3 * N + e] = l1;
    x[4 * N + e] = l2;
    if (t && un) {
        const double ue = u[e], pe = up ? up[e] : ue;
        t[e] = (float)((un[e] - 2.0 * ue + pe) * inv);
    }
}

__global__ void k_nn_pack_x(const float* __restrict__ x, bf16_t* __restrict__ out, NnDims d) {
    const long V1 = (long)d.D * d.H * d.W;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.vox()) return;
    const long b = i / V1, v = i - b * V1;
    const float* xb = x + b * kNnIn * V1;
    const float v0[4] = {xb[v], xb[V1 + v], xb[2 * V1 + v], xb[3 * V1 + v]};
    const float v1[4] = {xb[4 * V1 + v], 0.f, 0.f, 0.f};
    st4(out + i * 8, v0);
    st4(out + i * 8 + 4, v1);
}

__global__ void k_nn_crop(const float* __restrict__ src, int c, int nx, int ny, int nz, int x0,
                          int y0, int z0, int cx, int cy, int cz, float* __restrict__ dst) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)c * cz * cy * cx;
    if (i >= tot) return;
    const int x = (int)(i % cx);
    const int y = (int)((i / cx) % cy);
    const int z = (int)((i / ((long)cx * cy)) % cz);
    const int ch = (int)(i / ((long)cx * cy * cz));
    dst[i] = src[(((long)ch * nz + (z0 + z)) * ny + (y0 + y)) * nx + (x0 + x)];
}

__global__ __launch_bounds__(256) void k_nn_loss(const float* __restrict__ y,
                                                 const float* __restrict__ t, NnDims d, int margin,
                                                 double inv_cnt, bf16_t* __restrict__ gy,
                                                 double* __restrict__ partials) {
    __shared__ double sb[4];
    double acc = 0.0;
    const long V = d.vox();
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < V; i += (long)gridDim.x * 256) {
        int b, z, yy, x;
        unvox(i, d, b, z, yy, x);
        const bool in = z >= margin && z < d.D - margin && yy >= margin && yy < d.H - margin &&
                        x >= margin && x < d.W - margin;
        float g = 0.f;
        if (in) {
            const double r = (double)y[i] - (double)t[i];
            acc += r * r;
            g = (float)(2.0 * r * inv_cnt);
        }
        const float v[4] = {g, 0.f, 0.f, 0.f};
        st4(gy + i * 4, v);
    }
    const double S = nn_block_sum(acc, sb);
    if (threadIdx.x == 0) partials[blockIdx.x] = S;
}

__global__ __launch_bounds__(256) void k_nn_loss_fin(const double* __restrict__ partials, int np,
                                                     double inv_cnt, double* loss) {
    __shared__ double sb[4];
    double a = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) a += partials[i];
    const double S = nn_block_sum(a, sb);
    if (threadIdx.x == 0) *loss = S * inv_cnt;
}

__global__ void k_nn_head(const double* __restrict__ u, const double* __restrict__ up,
                          const float* __restrict__ y, const double* __restrict__ s, long N,
                          double* __restrict__ guess) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const double ue = u[e];
    guess[e] = ue + (up ? ue - up[e] : 0.0) + *s * (double)y[e];
}

__global__ void k_nn_adam(long n, float* __restrict__ p, const float* __restrict__ g,
                          float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                          float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

inline unsigned blocks(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t nn_frag(const float* W, int cin, int cout, int transposed, nn_s4* frag, int ks, int mb,
                   int kcin_p, hipStream_t s) {
    const long n = (long)ks * mb * 64;
    hipLaunchKernelGGL(k_nn_frag, dim3(blocks(n)), dim3(256), 0, s, W, cin, cout, transposed, frag,
                       ks, mb, kcin_p);
    return hipGetLastError();
}

hipError_t nn_conv(const NnConvArgs& a, int mb, hipStream_t s) {
    // z planes per workgroup: 4 for up to 32 input channels, 2 for 64 (LDS)
    const int R = a.cin_p <= 32 ? 4 : 2;
    const long nblk = (long)a.d.B * ((a.d.W + 15) / 16) * ((a.d.H + kConvTY - 1) / kConvTY) *
                      ((a.d.D + R - 1) / R);
    const size_t lds = (size_t)18 * (kConvTY + 2) * (R + 2) * (a.cin_p + 4) * sizeof(bf16_t);
    const dim3 g((unsigned)nblk);
#define NN_CONV_CASE(CP_, MB_, R_, K32_)                                                        \
    if (a.cin_p == CP_ && mb == MB_ && R == R_) {                                               \
        hipLaunchKernelGGL((k_nn_conv<CP_, MB_, R_, K32_>), g, dim3(256), lds, s, a);            \
        return hipGetLastError();                                                               \
    }
    // the (input pitch, output blocks) pairs of the network's forward and
    // input-gradient convolutions, with the MFMA shape measured faster at
    // 255^3 (K = 32 products where the pairing's extra registers cost no
    // occupancy: 251 against 261 us for 32 -> 16 channels, 112 against 116
    // and 43 against 57 us at 64 input channels; K = 16 elsewhere, e.g.
    // 441 against 498 us for 5 -> 16 channels)
    NN_CONV_CASE(8, 1, 4, false)
    NN_CONV_CASE(16, 2, 4, false)
    NN_CONV_CASE(32, 4, 4, false)
    NN_CONV_CASE(64, 4, 2, true)
    NN_CONV_CASE(64, 2, 2, true)
    NN_CONV_CASE(32, 1, 4, true)
    NN_CONV_CASE(16, 1, 4, false)
    NN_CONV_CASE(4, 1, 4, false)
#undef NN_CONV_CASE
    return hipErrorInvalidValue;
}

hipError_t nn_pool(const bf16_t* in, bf16_t* out, NnDims fine, NnDims coarse, int cp, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_pool, dim3(blocks(coarse.vox() * (cp / 4))), dim3(256), 0, s, in, out,
                       fine, coarse, cp);
    return hipGetLastError();
}

hipError_t nn_upadd(const bf16_t* coarse, const bf16_t* skip, bf16_t* out, NnDims fine,
                    NnDims c, int cp, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_upadd, dim3(blocks(fine.vox() * (cp / 4))), dim3(256), 0, s, coarse,
                       skip, out, fine, c, cp);
    return hipGetLastError();
}

hipError_t nn_up_bwd_mask(const bf16_t* gfine, const bf16_t* act, bf16_t* gcoarse, NnDims fine,
                          NnDims c, int cp, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_up_bwd_mask, dim3(blocks(c.vox() * (cp / 4))), dim3(256), 0, s, gfine,
                       act, gcoarse, fine, c, cp);
    return hipGetLastError();
}

hipError_t nn_pool_bwd_add_mask(const bf16_t* gcoarse, const bf16_t* gskip, const bf16_t* act,
                                bf16_t* g, NnDims fine, NnDims c, int cp, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_pool_bwd_add_mask, dim3(blocks(fine.vox() * (cp / 4))), dim3(256), 0, s,
                       gcoarse, gskip, act, g, fine, c, cp);
    return hipGetLastError();
}

long nn_wgrad_partials(const NnDims& d, int cin_p, int cout, int vchunk) {
    const long nchunks = (d.vox() + vchunk - 1) / vchunk;
    const int kn = (27 * cin_p + 15) / 16, mbn = (cout + 15) / 16;
    return nchunks * mbn * 16L * kn * 16L;
}

hipError_t nn_wgrad(const NnWgradArgs& a, hipStream_t s) {
    const long nchunks = (a.d.vox() + a.vchunk - 1) / a.vchunk;
    const int kn = (27 * a.cin_p + 15) / 16, mbn = (a.cout + 15) / 16;
    const long nwaves = nchunks * mbn * kn;
    hipLaunchKernelGGL(k_nn_wgrad, dim3(blocks(nwaves, 4)), dim3(256), 0, s, a, mbn, kn, nwaves);
    hipLaunchKernelGGL(k_nn_bgrad, dim3(blocks(nchunks * a.cout)), dim3(256), 0, s, a, nchunks);
    const long nr = (long)a.cout * a.cin * 27 + a.cout;
    hipLaunchKernelGGL(k_nn_wgrad_reduce, dim3(blocks(nr)), dim3(256), 0, s, a, mbn, kn, nchunks);
    return hipGetLastError();
}

hipError_t nn_scale(const double* u, const double* uprev, const double* F, const double* Fprev,
                    double dt, long N, double* partials, double* s_out, hipStream_t st) {
    long g = (N + 255) / 256;
    if (g > kNnGrid) g = kNnGrid;
    hipLaunchKernelGGL(k_nn_sumsq, dim3((unsigned)g), dim3(256), 0, st, u, uprev, F, Fprev, dt, N,
                       partials);
    hipLaunchKernelGGL(k_nn_scale_fin, dim3(1), dim3(256), 0, st, partials, (int)g, N, s_out);
    return hipGetLastError();
}

hipError_t nn_feat_bf16(const double* u, const double* uprev, const double* F, const double* Fprev,
                        double dt, const double* s, float l0, float l1, float l2, long N, bf16_t* x,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_nn_feat_bf16, dim3(blocks(N)), dim3(256), 0, st, u, uprev, F, Fprev, dt, s,
                       l0, l1, l2, N, x);
    return hipGetLastError();
}

hipError_t nn_feat_f32(const double* u, const double* uprev, const double* F, const double* Fprev,
                       const double* unext, double dt, const double* s, float l0, float l1,
                       float l2, long N, float* x, float* t, hipStream_t st) {
    hipLaunchKernelGGL(k_nn_feat_f32, dim3(blocks(N)), dim3(256), 0, st, u, uprev, F, Fprev, unext,
                       dt, s, l0, l1, l2, N, x, t);
    return hipGetLastError();
}

hipError_t nn_pack_x(const float* x, bf16_t* out, NnDims d, hipStream_t st) {
    hipLaunchKernelGGL(k_nn_pack_x, dim3(blocks(d.vox())), dim3(256), 0, st, x, out, d);
    return hipGetLastError();
}

hipError_t nn_crop(const float* src, int c, int nx, int ny, int nz, int x0, int y0, int z0, int cx,
                   int cy, int cz, float* dst, hipStream_t st) {
    const long tot = (long)c * cz * cy * cx;
    hipLaunchKernelGGL(k_nn_crop, dim3(blocks(tot)), dim3(256), 0, st, src, c, nx, ny, nz, x0, y0,
                       z0, cx, cy, cz, dst);
    return hipGetLastError();
}

hipError_t nn_loss(const float* y, const float* t, NnDims d, int margin, bf16_t* gy,
                   double* partials, double* loss, hipStream_t st) {
    const long cnt = (long)d.B * (d.D - 2 * margin) * (d.H - 2 * margin) * (d.W - 2 * margin);
    if (cnt <= 0) return hipErrorInvalidValue;
    long g = (d.vox() + 255) / 256;
    if (g > kNnGrid) g = kNnGrid;
    const double inv = 1.0 / (double)cnt;
    hipLaunchKernelGGL(k_nn_loss, dim3((unsigned)g), dim3(256), 0, st, y, t, d, margin, inv, gy,
                       partials);
    hipLaunchKernelGGL(k_nn_loss_fin, dim3(1), dim3(256), 0, st, partials, (int)g, inv, loss);
    return hipGetLastError();
}

hipError_t nn_head(const double* u, const double* uprev, const float* y, const double* s, long N,
                   double* guess, hipStream_t st) {
    hipLaunchKernelGGL(k_nn_head, dim3(blocks(N)), dim3(256), 0, st, u, uprev, y, s, N, guess);
    return hipGetLastError();
}

hipError_t nn_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1,
                   float b2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_nn_adam, dim3(blocks(n)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace fsd
