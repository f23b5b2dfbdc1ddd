// C ABI of the warm-start network (include/fsd_nn.h): workspace layout and
// the launch sequences of the forward pass, the backward pass and Adam.
#include <cmath>
#include <string>

#include "../../include/fsd_nn.h"
#include "fsd_host.h"
#include "fsd_nn.h"

using namespace fsd;

namespace {

#define NN_HIP(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_error(FSD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

constexpr int kVchunk = 1024;   // voxels per weight-gradient partial

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

struct LayerPlan {
    int cin, cout, cin_p, cout_p, level, relu;
    int ks, mb;            // forward: K-steps and 16-row output blocks
    int ksT, mbT;          // input gradient (transposed weights)
    long offW, offb;       // offsets in the flat parameter vector
};

}  // namespace

struct fsd_nn_s {
    int nx = 0, ny = 0, nz = 0, B = 1;
    bool training = false;
    NnDims lv[4];
    LayerPlan L[kNnLayers];
    long nparams = 0;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    hipStream_t stream = nullptr;
    // forward buffers (bf16 channels-last)
    bf16_t *x = nullptr, *e0 = nullptr, *p1 = nullptr, *e1 = nullptr, *p2 = nullptr, *e2 = nullptr,
           *p3 = nullptr, *e3 = nullptr, *s2 = nullptr, *d2 = nullptr, *s1 = nullptr, *d1 = nullptr,
           *s0 = nullptr;
    float* y32 = nullptr;
    nn_s4* frag[kNnLayers] = {};
    nn_s4* fragT[kNnLayers] = {};
    double* partials = nullptr;   // 2 * kNnGrid
    double* scal = nullptr;       // [0] = s
    // backward buffers
    bf16_t *gy = nullptr, *gs0 = nullptr, *gd1 = nullptr, *gs1 = nullptr, *gd2 = nullptr,
           *gs2 = nullptr, *ge3 = nullptr, *gp3 = nullptr, *ge2 = nullptr, *gp2 = nullptr,
           *ge1 = nullptr, *gp1 = nullptr, *ge0 = nullptr;
    float* wpart = nullptr;
    float* bpart = nullptr;
};

namespace {

NnDims coarse(const NnDims& d) { return NnDims{d.B, (d.D + 1) / 2, (d.H + 1) / 2, (d.W + 1) / 2}; }

struct Bump {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off = al256(off + count * sizeof(T));
        return p;
    }
};

size_t layout(fsd_nn nn, char* base) {
    Bump b{base};
    const NnDims* v = nn->lv;
    auto act = [&](int level, int c) { return b.take<bf16_t>((size_t)v[level].vox() * nn_pitch(c)); };
    nn->x = act(0, 8);
    nn->e0 = act(0, 16);
    nn->p1 = act(1, 16);
    nn->e1 = act(1, 32);
    nn->p2 = act(2, 32);
    nn->e2 = act(2, 64);
    nn->p3 = act(3, 64);
    nn->e3 = act(3, 64);
    nn->s2 = act(2, 64);
    nn->d2 = act(2, 32);
    nn->s1 = act(1, 32);
    nn->d1 = act(1, 16);
    nn->s0 = act(0, 16);
    nn->y32 = b.take<float>((size_t)v[0].vox());
    for (int k = 0; k < kNnLayers; ++k) {
        nn->frag[k] = b.take<nn_s4>((size_t)nn->L[k].ks * nn->L[k].mb * 64);
        nn->fragT[k] = b.take<nn_s4>((size_t)nn->L[k].ksT * nn->L[k].mbT * 64);
    }
    nn->partials = b.take<double>(2 * kNnGrid);
    nn->scal = b.take<double>(4);
    if (nn->training) {
        nn->gy = act(0, 1);
        nn->gs0 = act(0, 16);
        nn->gd1 = act(1, 16);
        nn->gs1 = act(1, 32);
        nn->gd2 = act(2, 32);
        nn->gs2 = act(2, 64);
        nn->ge3 = act(3, 64);
        nn->gp3 = act(3, 64);
        nn->ge2 = act(2, 64);
        nn->gp2 = act(2, 32);
        nn->ge1 = act(1, 32);
        nn->gp1 = act(1, 16);
        nn->ge0 = act(0, 16);
        long wp = 0, bp = 0;
        for (int k = 0; k < kNnLayers; ++k) {
            const NnDims& d = v[nn->L[k].level];
            const long n = nn_wgrad_partials(d, nn->L[k].cin_p, nn->L[k].cout, kVchunk);
            if (n > wp) wp = n;
            const long nb = ((d.vox() + kVchunk - 1) / kVchunk) * nn->L[k].cout;
            if (nb > bp) bp = nb;
        }
        nn->wpart = b.take<float>((size_t)wp);
        nn->bpart = b.take<float>((size_t)bp);
    }
    return b.off;
}

fsd_status check(fsd_nn nn) {
    if (!nn) return set_error(FSD_EINVAL, "null network");
    if (!nn->bound) return set_error(FSD_ENOTBOUND, "fsd_nn_bind() has not been called");
    return FSD_OK;
}

// A operands of every layer from the float32 parameters.
fsd_status build_frags(fsd_nn nn, const float* params, bool transposed) {
    for (int k = 0; k < kNnLayers; ++k) {
        const LayerPlan& l = nn->L[k];
        NN_HIP(nn_frag(params + l.offW, l.cin, l.cout, 0, nn->frag[k], l.ks, l.mb, l.cin_p,
                       nn->stream));
        if (transposed && k > 0)
            NN_HIP(nn_frag(params + l.offW, l.cin, l.cout, 1, nn->fragT[k], l.ksT, l.mbT, l.cout_p,
                           nn->stream));
    }
    return FSD_OK;
}

fsd_status conv(fsd_nn nn, int k, const bf16_t* in, bf16_t* out, float* out32,
                const float* params, const bf16_t* up = nullptr) {
    const LayerPlan& l = nn->L[k];
    NnConvArgs a{};
    a.in = in;
    a.up = up;
    if (up) a.upd = nn->lv[l.level + 1];
    a.cin_p = l.cin_p;
    a.cin_shift = nn_log2(l.cin_p);
    a.d = nn->lv[l.level];
    a.frag = nn->frag[k];
    a.ks = l.ks;
    a.bias = params + l.offb;
    a.cout = l.cout;
    a.out = out;
    a.cout_p = l.cout_p;
    a.out32 = out32;
    a.relu = l.relu;
    NN_HIP(nn_conv(a, l.mb, nn->stream));
    return FSD_OK;
}

// Input gradient of layer k: out (cin channels) = conv(gin (cout channels), W^T flipped).
fsd_status conv_t(fsd_nn nn, int k, const bf16_t* gin, bf16_t* gout) {
    const LayerPlan& l = nn->L[k];
    NnConvArgs a{};
    a.in = gin;
    a.cin_p = l.cout_p;
    a.cin_shift = nn_log2(l.cout_p);
    a.d = nn->lv[l.level];
    a.frag = nn->fragT[k];
    a.ks = l.ksT;
    a.bias = nullptr;
    a.cout = l.cin;
    a.out = gout;
    a.cout_p = l.cin_p;
    a.out32 = nullptr;
    a.relu = 0;
    NN_HIP(nn_conv(a, l.mbT, nn->stream));
    return FSD_OK;
}

fsd_status wgrad(fsd_nn nn, int k, const bf16_t* in, const bf16_t* gout, float* grad) {
    const LayerPlan& l = nn->L[k];
    NnWgradArgs a{};
    a.in = in;
    a.cin = l.cin;
    a.cin_p = l.cin_p;
    a.cin_shift = nn_log2(l.cin_p);
    a.gout = gout;
    a.cout = l.cout;
    a.cout_p = l.cout_p;
    a.d = nn->lv[l.level];
    a.vchunk = kVchunk;
    a.partials = nn->wpart;
    a.bpartials = nn->bpart;
    a.gW = grad + l.offW;
    a.gb = grad + l.offb;
    NN_HIP(nn_wgrad(a, nn->stream));
    return FSD_OK;
}

#define NN_TRY(expr)                    \
    do {                                \
        fsd_status s_ = (expr);         \
        if (s_ != FSD_OK) return s_;    \
    } while (0)

// Forward pass from nn->x.  A training instance materialises every
// activation (the backward pass reads them); an inference instance fuses
// each decoder upsample-and-add into the staging of the next convolution.
fsd_status forward(fsd_nn nn, const float* params) {
    hipStream_t s = nn->stream;
    const NnDims* v = nn->lv;
    const bool keep = nn->training;
    NN_TRY(conv(nn, 0, nn->x, nn->e0, nullptr, params));
    NN_HIP(nn_pool(nn->e0, nn->p1, v[0], v[1], 16, s));
    NN_TRY(conv(nn, 1, nn->p1, nn->e1, nullptr, params));
    NN_HIP(nn_pool(nn->e1, nn->p2, v[1], v[2], 32, s));
    NN_TRY(conv(nn, 2, nn->p2, nn->e2, nullptr, params));
    NN_HIP(nn_pool(nn->e2, nn->p3, v[2], v[3], 64, s));
    NN_TRY(conv(nn, 3, nn->p3, nn->e3, nullptr, params));
    if (keep) {
        NN_HIP(nn_upadd(nn->e3, nn->e2, nn->s2, v[2], v[3], 64, s));
        NN_TRY(conv(nn, 4, nn->s2, nn->d2, nullptr, params));
        NN_HIP(nn_upadd(nn->d2, nn->e1, nn->s1, v[1], v[2], 32, s));
        NN_TRY(conv(nn, 5, nn->s1, nn->d1, nullptr, params));
        NN_HIP(nn_upadd(nn->d1, nn->e0, nn->s0, v[0], v[1], 16, s));
        NN_TRY(conv(nn, 6, nn->s0, nullptr, nn->y32, params));
    } else {
        NN_TRY(conv(nn, 4, nn->e2, nn->d2, nullptr, params, nn->e3));
        NN_TRY(conv(nn, 5, nn->e1, nn->d1, nullptr, params, nn->d2));
        NN_TRY(conv(nn, 6, nn->e0, nullptr, nn->y32, params, nn->d1));
    }
    return FSD_OK;
}

fsd_status backward(fsd_nn nn, float* grad) {
    hipStream_t s = nn->stream;
    const NnDims* v = nn->lv;
    // d0 (level 0): input s0 = up(d1) + e0
    NN_TRY(conv_t(nn, 6, nn->gy, nn->gs0));
    NN_TRY(wgrad(nn, 6, nn->s0, nn->gy, grad));
    NN_HIP(nn_up_bwd_mask(nn->gs0, nn->d1, nn->gd1, v[0], v[1], 16, s));
    // d1 (level 1): input s1 = up(d2) + e1
    NN_TRY(conv_t(nn, 5, nn->gd1, nn->gs1));
    NN_TRY(wgrad(nn, 5, nn->s1, nn->gd1, grad));
    NN_HIP(nn_up_bwd_mask(nn->gs1, nn->d2, nn->gd2, v[1], v[2], 32, s));
    // d2 (level 2): input s2 = up(e3) + e2
    NN_TRY(conv_t(nn, 4, nn->gd2, nn->gs2));
    NN_TRY(wgrad(nn, 4, nn->s2, nn->gd2, grad));
    NN_HIP(nn_up_bwd_mask(nn->gs2, nn->e3, nn->ge3, v[2], v[3], 64, s));
    // e3 (level 3): input p3 = pool(e2)
    NN_TRY(conv_t(nn, 3, nn->ge3, nn->gp3));
    NN_TRY(wgrad(nn, 3, nn->p3, nn->ge3, grad));
    NN_HIP(nn_pool_bwd_add_mask(nn->gp3, nn->gs2, nn->e2, nn->ge2, v[2], v[3], 64, s));
    // e2 (level 2): input p2 = pool(e1)
    NN_TRY(conv_t(nn, 2, nn->ge2, nn->gp2));
    NN_TRY(wgrad(nn, 2, nn->p2, nn->ge2, grad));
    NN_HIP(nn_pool_bwd_add_mask(nn->gp2, nn->gs1, nn->e1, nn->ge1, v[1], v[2], 32, s));
    // e1 (level 1): input p1 = pool(e0)
    NN_TRY(conv_t(nn, 1, nn->ge1, nn->gp1));
    NN_TRY(wgrad(nn, 1, nn->p1, nn->ge1, grad));
    NN_HIP(nn_pool_bwd_add_mask(nn->gp1, nn->gs0, nn->e0, nn->ge0, v[0], v[1], 16, s));
    // e0 (level 0): input x
    NN_TRY(wgrad(nn, 0, nn->x, nn->ge0, grad));
    return FSD_OK;
}

}  // namespace

extern "C" {

long fsd_nn_param_count(void) {
    long n = 0;
    for (int k = 0; k < kNnLayers; ++k) n += (long)kNnLayer[k].cout * kNnLayer[k].cin * 27 + kNnLayer[k].cout;
    return n;
}

fsd_status fsd_nn_layer(int k, int* c_in, int* c_out, int* level) {
    if (k < 0 || k >= kNnLayers) return set_error(FSD_EINVAL, "layer index outside [0, 6]");
    if (c_in) *c_in = kNnLayer[k].cin;
    if (c_out) *c_out = kNnLayer[k].cout;
    if (level) *level = kNnLayer[k].level;
    return FSD_OK;
}

fsd_status fsd_nn_create(int nx, int ny, int nz, int batch, int training, fsd_nn* out) {
    if (!out) return set_error(FSD_EINVAL, "null output handle");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1 || batch < 1)
        return set_error(FSD_EINVAL, "grid sizes and batch must be >= 1");
    if ((long)nx * ny * nz * batch > (1L << 31) / 16)
        return set_error(FSD_EINVAL, "grid too large for the network");
    fsd_nn nn = new fsd_nn_s();
    nn->nx = nx;
    nn->ny = ny;
    nn->nz = nz;
    nn->B = batch;
    nn->training = training != 0;
    nn->lv[0] = NnDims{batch, nz, ny, nx};
    for (int l = 1; l < 4; ++l) nn->lv[l] = coarse(nn->lv[l - 1]);
    long off = 0;
    for (int k = 0; k < kNnLayers; ++k) {
        LayerPlan& p = nn->L[k];
        p.cin = kNnLayer[k].cin;
        p.cout = kNnLayer[k].cout;
        p.level = kNnLayer[k].level;
        p.relu = kNnLayer[k].relu;
        p.cin_p = k == 0 ? 8 : nn_pitch(p.cin);
        p.cout_p = nn_pitch(p.cout);
        p.ks = (27 * p.cin_p + 15) / 16;
        p.mb = (p.cout + 15) / 16;
        if (p.mb == 3) p.mb = 4;
        p.ksT = (27 * p.cout_p + 15) / 16;
        p.mbT = (p.cin + 15) / 16;
        if (p.mbT == 3) p.mbT = 4;
        p.offW = off;
        off += (long)p.cout * p.cin * 27;
        p.offb = off;
        off += p.cout;
    }
    nn->nparams = off;
    nn->ws_bytes = layout(nn, nullptr);
    *out = nn;
    return FSD_OK;
}

void fsd_nn_destroy(fsd_nn nn) { delete nn; }

size_t fsd_nn_workspace_bytes(fsd_nn nn) { return nn ? nn->ws_bytes : 0; }

fsd_status fsd_nn_bind(fsd_nn nn, void* d_ws, size_t bytes, void* stream) {
    if (!nn || !d_ws) return set_error(FSD_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(d_ws) % 256) return set_error(FSD_EINVAL, "workspace not 256-byte aligned");
    if (bytes < nn->ws_bytes) return set_error(FSD_ESMALLWS, "workspace smaller than fsd_nn_workspace_bytes()");
    nn->ws = static_cast<char*>(d_ws);
    nn->stream = static_cast<hipStream_t>(stream);
    layout(nn, nn->ws);
    nn->bound = true;
    return FSD_OK;
}

fsd_status fsd_nn_features(fsd_nn nn, const double* d_u, const double* d_uprev, const double* d_F,
                           const double* d_Fprev, const double* d_unext, double dt,
                           const double eta[3], float* d_x, float* d_t, double* d_s) {
    NN_TRY(check(nn));
    if (!d_u || !d_x || !eta) return set_error(FSD_EINVAL, "null argument");
    for (int i = 0; i < 3; ++i)
        if (!(eta[i] > 0.0)) return set_error(FSD_EINVAL, "eta must be positive");
    const long N = (long)nn->nx * nn->ny * nn->nz;
    NN_HIP(nn_scale(d_u, d_uprev, d_F, d_Fprev, dt, N, nn->partials, nn->scal, nn->stream));
    NN_HIP(nn_feat_f32(d_u, d_uprev, d_F, d_Fprev, d_unext, dt, nn->scal,
                       (float)(std::log(eta[0]) / 4), (float)(std::log(eta[1]) / 4),
                       (float)(std::log(eta[2]) / 4), N, d_x, d_t, nn->stream));
    if (d_s) NN_HIP(hipMemcpyAsync(d_s, nn->scal, sizeof(double), hipMemcpyDeviceToDevice, nn->stream));
    return FSD_OK;
}

fsd_status fsd_nn_crop(const float* d_src, int c, int nx, int ny, int nz, int x0, int y0, int z0,
                       int cx, int cy, int cz, float* d_dst, void* stream) {
    if (!d_src || !d_dst) return set_error(FSD_EINVAL, "null argument");
    if (c < 1 || cx < 1 || cy < 1 || cz < 1 || x0 < 0 || y0 < 0 || z0 < 0 || x0 + cx > nx ||
        y0 + cy > ny || z0 + cz > nz)
        return set_error(FSD_EINVAL, "crop box outside the grid");
    NN_HIP(nn_crop(d_src, c, nx, ny, nz, x0, y0, z0, cx, cy, cz, d_dst,
                   static_cast<hipStream_t>(stream)));
    return FSD_OK;
}

fsd_status fsd_nn_forward(fsd_nn nn, const float* d_params, const float* d_x, float* d_y) {
    NN_TRY(check(nn));
    if (!d_params || !d_x || !d_y) return set_error(FSD_EINVAL, "null argument");
    NN_TRY(build_frags(nn, d_params, false));
    NN_HIP(nn_pack_x(d_x, nn->x, nn->lv[0], nn->stream));
    NN_TRY(forward(nn, d_params));
    NN_HIP(hipMemcpyAsync(d_y, nn->y32, sizeof(float) * nn->lv[0].vox(), hipMemcpyDeviceToDevice,
                          nn->stream));
    return FSD_OK;
}

fsd_status fsd_nn_loss_grad(fsd_nn nn, const float* d_params, const float* d_x, const float* d_t,
                            int margin, float* d_grad, double* d_loss) {
    NN_TRY(check(nn));
    if (!nn->training) return set_error(FSD_EINVAL, "not a training instance");
    if (!d_params || !d_x || !d_t || !d_grad || !d_loss) return set_error(FSD_EINVAL, "null argument");
    const NnDims& d = nn->lv[0];
    if (margin < 0 || 2 * margin >= d.D || 2 * margin >= d.H || 2 * margin >= d.W)
        return set_error(FSD_EINVAL, "margin leaves no interior");
    NN_TRY(build_frags(nn, d_params, true));
    NN_HIP(nn_pack_x(d_x, nn->x, d, nn->stream));
    NN_TRY(forward(nn, d_params));
    NN_HIP(nn_loss(nn->y32, d_t, d, margin, nn->gy, nn->partials, d_loss, nn->stream));
    NN_TRY(backward(nn, d_grad));
    return FSD_OK;
}

fsd_status fsd_nn_adam(long count, float* d_p, const float* d_g, float* d_m, float* d_v, int t,
                       double lr, double b1, double b2, double eps, void* stream) {
    if (!d_p || !d_g || !d_m || !d_v || count < 1 || t < 1)
        return set_error(FSD_EINVAL, "bad Adam arguments");
    const double c1 = 1.0 / (1.0 - std::pow(b1, t)), c2 = 1.0 / (1.0 - std::pow(b2, t));
    NN_HIP(nn_adam(count, d_p, d_g, d_m, d_v, (float)lr, (float)b1, (float)b2, (float)eps, (float)c1,
                   (float)c2, static_cast<hipStream_t>(stream)));
    return FSD_OK;
}

fsd_status fsd_nn_predict(fsd_nn nn, const float* d_params, const double* d_u,
                          const double* d_uprev, const double* d_F, const double* d_Fprev,
                          double dt, const double eta[3], double* d_guess) {
    NN_TRY(check(nn));
    if (!d_params || !d_u || !d_guess || !eta) return set_error(FSD_EINVAL, "null argument");
    if (nn->B != 1) return set_error(FSD_EINVAL, "prediction needs a batch-1 instance");
    for (int i = 0; i < 3; ++i)
        if (!(eta[i] > 0.0)) return set_error(FSD_EINVAL, "eta must be positive");
    const long N = (long)nn->nx * nn->ny * nn->nz;
    hipStream_t s = nn->stream;
    NN_TRY(build_frags(nn, d_params, false));
    NN_HIP(nn_scale(d_u, d_uprev, d_F, d_Fprev, dt, N, nn->partials, nn->scal, s));
    NN_HIP(nn_feat_bf16(d_u, d_uprev, d_F, d_Fprev, dt, nn->scal, (float)(std::log(eta[0]) / 4),
                        (float)(std::log(eta[1]) / 4), (float)(std::log(eta[2]) / 4), N, nn->x, s));
    NN_TRY(forward(nn, d_params));
    NN_HIP(nn_head(d_u, d_uprev, nn->y32, nn->scal, N, d_guess, s));
    return FSD_OK;
}

}  // extern "C"
