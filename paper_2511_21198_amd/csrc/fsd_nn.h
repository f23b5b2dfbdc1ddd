// Internal declarations of the warm-start network kernels (fsd_nn.hip).
//
// Activations are bfloat16, channels-last ([batch][z][y][x][c], c fastest)
// with a channel pitch that is a multiple of 4, so that four consecutive
// channels of one voxel are one 8-byte load: that is the K-slice one lane
// feeds to a 16x16x16 bf16 MFMA, or to one half of a 16x16x32 one (two
// 16-value K steps per instruction).  Accumulation is float32.
#pragma once

#include <hip/hip_runtime.h>

namespace fsd {

typedef unsigned short bf16_t;
typedef short nn_s4 __attribute__((ext_vector_type(4)));

struct NnLayer {
    int cin, cout, level, relu;
};
constexpr int kNnLayers = 7;
constexpr int kNnIn = 5;
// e0 e1 e2 e3 d2 d1 d0 (the order of the flat parameter vector)
constexpr NnLayer kNnLayer[kNnLayers] = {
    {5, 16, 0, 1}, {16, 32, 1, 1}, {32, 64, 2, 1}, {64, 64, 3, 1},
    {64, 32, 2, 1}, {32, 16, 1, 1}, {16, 1, 0, 0},
};

// Channel pitch of a tensor with c channels: a power of two >= 4.
constexpr int nn_pitch(int c) { return c <= 4 ? 4 : c <= 8 ? 8 : c <= 16 ? 16 : c <= 32 ? 32 : 64; }
constexpr int nn_log2(int v) { return v <= 1 ? 0 : 1 + nn_log2(v / 2); }

struct NnDims {
    int B, D, H, W;
    __host__ __device__ long vox() const { return (long)B * D * H * W; }
};

// 3x3x3 convolution (zero padding, stride 1) as an implicit GEMM on MFMA.
// out[v][o] = bias[o] + sum_{tap, i} frag(o, tap, i) * in[v + off(tap)][i],
// K index k = tap * cin_p + i (27 taps, cin_p channels), ks = ceil(27 cin_p / 16)
// K-steps of 16 (one per 16x16x16 MFMA or two per 16x16x32 MFMA, by layer
// shape).  frag holds the A operands:
// [ks][mb][64 lanes] x 4 bf16.
struct NnConvArgs {
    const bf16_t* in;
    int cin_p, cin_shift;
    NnDims d;
    const nn_s4* frag;
    int ks;
    const float* bias;   // may be null
    int cout;            // channels written with values (others zero)
    bf16_t* out;         // may be null
    int cout_p;
    float* out32;        // channel 0 as float32 [voxel] (may be null)
    int relu;
    const bf16_t* up;    // optional: input is in[v] + up[v / 2] (pitch cin_p)
    NnDims upd;          // dimensions of `up`
};

// A operands of a layer.  transposed = 0: rows o < cout, K = (tap, i < cin)
// from W[o][i][tap].  transposed = 1 (input gradient): rows i < cin, K =
// (tap, o < cout) from W[o][i][26 - tap].
hipError_t nn_frag(const float* W, int cin, int cout, int transposed, nn_s4* frag, int ks, int mb,
                   int kcin_p, hipStream_t s);
hipError_t nn_conv(const NnConvArgs& a, int mb, hipStream_t s);

hipError_t nn_pool(const bf16_t* in, bf16_t* out, NnDims fine, NnDims coarse, int cp, hipStream_t s);
hipError_t nn_upadd(const bf16_t* coarse, const bf16_t* skip, bf16_t* out, NnDims fine,
                    NnDims c, int cp, hipStream_t s);
// g_coarse = (sum of the fine gradients over each 2x2x2 block) * (act > 0)
hipError_t nn_up_bwd_mask(const bf16_t* gfine, const bf16_t* act, bf16_t* gcoarse, NnDims fine,
                          NnDims coarse, int cp, hipStream_t s);
// g = (gskip + gcoarse[v/2] / 8) * (act > 0) on the fine grid
hipError_t nn_pool_bwd_add_mask(const bf16_t* gcoarse, const bf16_t* gskip, const bf16_t* act,
                                bf16_t* g, NnDims fine, NnDims coarse, int cp, hipStream_t s);

// Weight gradient of one layer: per chunk of `vchunk` voxels, the partial
// sums dW[o][k] = sum_v gout[v][o] in[v + off(tap)][i] (k = tap cin_p + i),
// then a fixed-order reduction over chunks into gW[o][i][tap] and gb[o].
struct NnWgradArgs {
    const bf16_t* in;
    int cin, cin_p, cin_shift;
    const bf16_t* gout;
    int cout, cout_p;
    NnDims d;
    int vchunk;
    float* partials;     // [nchunks][mb*16][kn*16]
    float* bpartials;    // [nchunks][cout]
    float* gW;           // [cout][cin][27]
    float* gb;           // [cout]
};
long nn_wgrad_partials(const NnDims& d, int cin_p, int cout, int vchunk);
hipError_t nn_wgrad(const NnWgradArgs& a, hipStream_t s);

// Features on the full grid (dense float64, x fastest): du = u - uprev,
// df = dt (F - Fprev), channels [du, df, l0, l1, l2] / s (the last three
// constant) with s = rms(du) + rms(df) + 1e-30 reduced on the device into
// *s_out.  Null uprev: du = 0; null F or Fprev: zero source.
hipError_t nn_scale(const double* u, const double* uprev, const double* F, const double* Fprev,
                    double dt, long N, double* partials, double* s_out, hipStream_t st);
hipError_t nn_feat_bf16(const double* u, const double* uprev, const double* F, const double* Fprev,
                        double dt, const double* s, float l0, float l1, float l2, long N, bf16_t* x,
                        hipStream_t st);
// float32 channels-first; t = (unext - 2 u + uprev) / s when unext is given.
hipError_t nn_feat_f32(const double* u, const double* uprev, const double* F, const double* Fprev,
                       const double* unext, double dt, const double* s, float l0, float l1,
                       float l2, long N, float* x, float* t, hipStream_t st);
// float32 [B][5][D][H][W] -> bf16 [B][D][H][W][8]
hipError_t nn_pack_x(const float* x, bf16_t* out, NnDims d, hipStream_t st);
hipError_t nn_crop(const float* src, int c, int nx, int ny, int nz, int x0, int y0, int z0, int cx,
                   int cy, int cz, float* dst, hipStream_t st);
// loss = mean over the interior of (y - t)^2; gy[v][0] = 2 (y - t) / count there, 0 elsewhere.
hipError_t nn_loss(const float* y, const float* t, NnDims d, int margin, bf16_t* gy,
                   double* partials, double* loss, hipStream_t st);
// guess = u + (u - uprev) + s * y  (uprev == null: guess = u + s * y)
hipError_t nn_head(const double* u, const double* uprev, const float* y, const double* s, long N,
                   double* guess, hipStream_t st);
hipError_t nn_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1,
                   float b2, float eps, float c1, float c2, hipStream_t st);

constexpr int kNnGrid = 1024;   // reduction grid of the feature scale and the loss

}  // namespace fsd
