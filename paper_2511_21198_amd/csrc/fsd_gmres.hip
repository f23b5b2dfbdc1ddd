// Kernels of the left-preconditioned restarted GMRES (Section 3.2,
// ``one_side_system``): Arnoldi on w = P^{-1} A v_j with classical
// Gram-Schmidt applied twice (CGS2), Givens rotations on the small
// Hessenberg matrix held in device memory (one thread), and the final
// update x += V y.
//
// Memory traffic per Arnoldi step j (nv = j + 1 basis vectors):
//   k_mdot      reads V[0..j], w                 -> partials of V^T w
//   k_maxpy     reads V[0..j], w, writes w       -> w -= V h1, partials of V^T w
//   k_maxpy     reads V[0..j], w, writes v_{j+1} -> w -= V h2, partial ||w||^2
// Each kernel loads the nv basis values of an element once into registers.
//
// With one Gram-Schmidt pass (zero reorthogonalisation threshold) and the
// wave engine's x pass, the update of v_{j+1} moves into the prologue of the
// next matvec (PRO_ARNOLDI): that x pass reads w and V[0..j], writes the new
// basis vector and the partials of its norm, and transforms it, which saves
// the k_maxpy launch and two vector passes per step.  The basis is then kept
// unnormalised (V_i = v_i / s_i, the scales in ctrl->gm): GM_COEF turns the
// multi-dot into the Hessenberg column and the prologue's coefficients,
// GM_NEXT the norm into H[j+1, j] and the Givens step, and GM_SOLVE folds the
// scales into y.
#include "fsd_gmres.h"

namespace fsd {

namespace {

constexpr int GT = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the workgroup; valid in thread 0.  sbuf holds GT/64 doubles.
__device__ inline double block_sum(double v, double* sbuf) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sbuf[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < GT / 64; ++i) s += sbuf[i];
    }
    return s;
}

// Block sums of nv per-thread accumulators with one workgroup barrier:
// wavefront reduction of each value, then one thread per value adds the
// wavefront results in order.  Writes partials[i * gridDim.x + blockIdx.x].
template <int NVMAX>
__device__ inline void block_multi_sum(const double (&acc)[NVMAX], int nv, double* red,
                                       double* __restrict__ partials) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) {
        if (i < nv) {
            const double v = wave_sum(acc[i]);
            if (lane == 0) red[w * NVMAX + i] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < GT / 64; ++k) s += red[k * NVMAX + threadIdx.x];
        partials[(long)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

// 16-byte vector of T: each lane moves 16 bytes per load (float4 / double2).
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int W = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int W = 2; };

template <typename V>
__device__ inline double vdot(const V& a, const V& b);
template <>
__device__ inline double vdot<float4>(const float4& a, const float4& b) {
    // products of floats are exact in double
    return ((double)a.x * (double)b.x + (double)a.y * (double)b.y) +
           ((double)a.z * (double)b.z + (double)a.w * (double)b.w);
}
template <>
__device__ inline double vdot<double2>(const double2& a, const double2& b) {
    return a.x * b.x + a.y * b.y;
}
template <typename T, typename V>
__device__ inline void vfms(V& o, T h, const V& v) {   // o -= h v
    o.x -= h * v.x; o.y -= h * v.y;
    if constexpr (sizeof(V) / sizeof(T) == 4) { o.z -= h * v.z; o.w -= h * v.w; }
}
template <typename T, typename V>
__device__ inline void vfma(V& o, T h, const V& v) {   // o += h v
    o.x += h * v.x; o.y += h * v.y;
    if constexpr (sizeof(V) / sizeof(T) == 4) { o.z += h * v.z; o.w += h * v.w; }
}

// Like block_multi_sum for nv + 1 values: acc[0..nv-1] to rows 0..nv-1 and
// the extra accumulator acc[NVMAX] to row nv.
template <int NVMAX>
__device__ inline void block_multi_sum_ext(const double (&acc)[NVMAX + 1], int nv, double* red,
                                           double* __restrict__ partials) {
    constexpr int NR = NVMAX + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i < nv || i == NVMAX) {
            const double v = wave_sum(acc[i]);
            if (lane == 0) red[w * NR + i] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x <= nv) {
        const int src = threadIdx.x < nv ? threadIdx.x : NVMAX;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < GT / 64; ++k) s += red[k * NR + src];
        partials[(long)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

// The vector kernels are instantiated for every basis size NV up to
// kExactNV (EXACT = true: the loops over the basis are fully unrolled with no
// predicates, so all NV + 1 loads of an iteration are in flight together) and
// once generically (NV = kMaxRestart + 1, predicated on the runtime count).
// N is a multiple of the vector width (the padded layout rounds the x extent
// up to 32) and every vector is 256-byte aligned.

// Arnoldi on P^{-1} A - I.  The preconditioned operator is close to the
// identity (Theorem 3.1), so w = P^{-1} A v_j is dominated by v_j, and
// Gram-Schmidt on w itself cancels that component with an absolute rounding
// error of about eps ||w||, far above ||w - V V^T w||: a second pass is then
// always needed.  Subtracting v_j first (w - v_j is exact where w and v_j
// agree to a factor of 2) leaves a vector the projection does not cancel,
// and one pass usually passes the reorthogonalisation test.  The Krylov
// space is the same; the Hessenberg column gets 1 added on its diagonal.
//
// partials[i * G + blk] = sum_e V_i[e] (w[e] - V_{nv-1}[e]) for i < nv, and
// row nv the partial ||w - V_{nv-1}||^2 (the reference of the test).
template <typename T, int NV, bool EXACT>
__global__ __launch_bounds__(GT) void k_mdot(const T* __restrict__ V, long ld, int nv_rt,
                                             const T* __restrict__ w, long N,
                                             double* __restrict__ partials, const Ctrl* ctrl) {
    using VT = typename Vec16<T>::type;
    constexpr int VW = Vec16<T>::W;
    __shared__ double red[(GT / 64) * (NV + 1)];
    if (ctrl->done) return;
    const int nv = EXACT ? NV : nv_rt;
    double acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    const long NW = N / VW, ldw = ld / VW;
    const VT* __restrict__ Vv = reinterpret_cast<const VT*>(V);
    const VT* __restrict__ wv = reinterpret_cast<const VT*>(w);
    const VT* __restrict__ vj = Vv + (long)(nv - 1) * ldw;
    for (long e = blockIdx.x * (long)GT + threadIdx.x; e < NW; e += (long)gridDim.x * GT) {
        VT we = wv[e];
        vfms<T>(we, T(1), vj[e]);
        VT v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) v[i] = Vv[i * ldw + e];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) acc[i] += vdot(v[i], we);
        acc[NV] += vdot(we, we);
    }
    block_multi_sum_ext<NV>(acc, nv, red, partials);
}

// out = in - sum_i h_i V_i (h from ctrl->gm + hoff), then
//   mode MX_DOTS:   out = in - V_{nv-1} - sum_i h_i V_i (the shifted first
//                   Gram-Schmidt pass, see k_mdot), partial dots V_i^T out
//                   (rows < nv) and ||out||^2 (row nv);
//   mode MX_NORM:   partial ||out||^2;
//   mode MX_REORTH: as MX_NORM, but only when ctrl->gm_reorth is set (the
//                   second Gram-Schmidt pass); otherwise nothing.
template <typename T, int NV, bool EXACT>
__global__ __launch_bounds__(GT) void k_maxpy(const T* __restrict__ V, long ld, int nv_rt,
                                              const T* in, T* out, long N, const Ctrl* ctrl,
                                              int hoff, int mode, double* __restrict__ partials) {
    using VT = typename Vec16<T>::type;
    constexpr int VW = Vec16<T>::W;
    __shared__ double sb[GT / 64];
    __shared__ double red[(GT / 64) * (NV + 1)];
    if (ctrl->done) return;
    if (mode == MX_REORTH && !ctrl->gm_reorth) return;
    const bool dots = mode == MX_DOTS;
    const int nv = EXACT ? NV : nv_rt;
    T h[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) h[i] = i < nv ? (T)ctrl->gm[hoff + i] : T(0);
    double acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    const long NW = N / VW, ldw = ld / VW;
    const VT* __restrict__ Vv = reinterpret_cast<const VT*>(V);
    const VT* inv = reinterpret_cast<const VT*>(in);
    VT* outv = reinterpret_cast<VT*>(out);
    const VT* __restrict__ vj = Vv + (long)(nv - 1) * ldw;
    // k_mdot has just swept the same vectors from the front; sweeping from the
    // back first reads what the caches still hold (5% faster in isolation)
    for (long e0 = blockIdx.x * (long)GT + threadIdx.x; e0 < NW; e0 += (long)gridDim.x * GT) {
        const long e = NW - 1 - e0;
        VT o = inv[e];
        if (dots) vfms<T>(o, T(1), vj[e]);   // exact where in and v_j agree to a factor 2
        VT v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) v[i] = Vv[i * ldw + e];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) vfms<T>(o, h[i], v[i]);
        outv[e] = o;
        if (dots) {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i < nv) acc[i] += vdot(v[i], o);
        }
        acc[NV] += vdot(o, o);
    }
    if (dots) {
        block_multi_sum_ext<NV>(acc, nv, red, partials);
    } else {
        const double s = block_sum(acc[NV], sb);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

// x += sum_{i < k} y_i V_i with k = ctrl->gm_k and y in ctrl->gm (yoff);
// with overwrite, x = sum_{i < k} y_i V_i (x = 0 for k = 0; x is not read).
// The host launches the instance NV = k; any other k (k = 0 after an
// immediate convergence) takes the predicated loop, which never touches a
// basis vector beyond k (unwritten memory may hold NaN patterns).
template <typename T, int NV, bool EXACT>
__global__ __launch_bounds__(GT) void k_gm_update(T* x, const T* __restrict__ V, long ld, long N,
                                                  const Ctrl* ctrl, int yoff, int overwrite) {
    using VT = typename Vec16<T>::type;
    constexpr int VW = Vec16<T>::W;
    const int k = ctrl->gm_k;
    if (k <= 0 && !overwrite) return;
    T y[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) y[i] = i < k ? (T)ctrl->gm[yoff + i] : T(0);
    const long NW = N / VW, ldw = ld / VW;
    const VT* __restrict__ Vv = reinterpret_cast<const VT*>(V);
    VT* xv = reinterpret_cast<VT*>(x);
    const bool full = EXACT && k == NV;
    for (long e = blockIdx.x * (long)GT + threadIdx.x; e < NW; e += (long)gridDim.x * GT) {
        VT acc;
        if (overwrite) {
            acc.x = T(0); acc.y = T(0);
            if constexpr (VW == 4) { acc.z = T(0); acc.w = T(0); }
        } else {
            acc = xv[e];
        }
        VT v[NV];
        if (full) {
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] = Vv[i * ldw + e];
#pragma unroll
            for (int i = 0; i < NV; ++i) vfma<T>(acc, y[i], v[i]);
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i < k) vfma<T>(acc, y[i], Vv[i * ldw + e]);
        }
        xv[e] = acc;
    }
}

// out = ctrl->gm_scale * in
template <typename T>
__global__ __launch_bounds__(GT) void k_scale(const T* in, T* out, long N, const Ctrl* ctrl) {
    if (ctrl->done) return;
    const T s = (T)ctrl->gm_scale;
    for (long e = blockIdx.x * (long)GT + threadIdx.x; e < N; e += (long)gridDim.x * GT)
        out[e] = s * in[e];
}

// v_cmp_class based; an arithmetic test such as v - v == 0 is unsound under
// FP contraction (the subtraction can fuse with the multiply producing v).
__device__ inline bool gm_isfinite(double v) { return __builtin_isfinite(v); }

// Scalar GMRES steps (one workgroup).
// Layout of ctrl->gm for restart m: H (m+1) x m column-major at 0,
// cs at GM_CS, sn at GM_SN, g at GM_G (m+1), y at GM_Y (m), h2 at GM_T (m+1),
// basis scales s at GM_T + m + 1 (m + 1).
// The partial sums of each value are added by one or more wavefronts in a
// fixed order (a row of many partials is split over several wavefronts).
// Per-row work runs one thread per row; the serial recurrences (Givens
// rotations, back substitution) run on thread 0 over copies staged in LDS,
// since thread 0 reading device memory it has just written would wait for
// each store.
constexpr int ST = 1024;
constexpr int SNW = ST / 64;

// Column j of the Hessenberg matrix is complete up to H[j+1, j] = hnext:
// apply the earlier rotations, form the new one, update g and test.  Called
// by every thread of the workgroup.
__device__ inline void gm_givens(Ctrl* c, double* gm, int m, int j, double hnext, double* sH,
                                 double* sCS, double* sSN) {
    const int oCS = (m + 1) * m, oSN = oCS + m, oG = oSN + m;
    const int tid = threadIdx.x;
    double* H = gm + (m + 1) * j;   // column j
    if (tid <= j) sH[tid] = H[tid];
    if (tid < j) { sCS[tid] = gm[oCS + tid]; sSN[tid] = gm[oSN + tid]; }
    __syncthreads();
    if (tid != 0) return;
    const double gj = gm[oG + j];
    sH[j + 1] = hnext;
    for (int i = 0; i < j; ++i) {
        const double cs = sCS[i], sn = sSN[i];
        const double t = cs * sH[i] + sn * sH[i + 1];
        sH[i + 1] = -sn * sH[i] + cs * sH[i + 1];
        sH[i] = t;
    }
    const double den = hypot(sH[j], sH[j + 1]);
    double cs = 1.0, sn = 0.0;
    if (den > 0.0) { cs = sH[j] / den; sn = sH[j + 1] / den; }
    sH[j] = den;
    sH[j + 1] = 0.0;
    for (int i = 0; i <= j + 1; ++i) H[i] = sH[i];
    gm[oCS + j] = cs;
    gm[oSN + j] = sn;
    const double res = -sn * gj;
    gm[oG + j + 1] = res;
    gm[oG + j] = cs * gj;
    c->iters += 1;
    c->gm_k = j + 1;
    c->gm_j = j + 1;
    c->rr = res * res;
    c->gm_hnext = hnext;
    c->gm_scale = hnext > 0.0 ? 1.0 / hnext : 0.0;
    if (!gm_isfinite(res)) { c->status = 4; c->done = 1; }
    else if (res * res <= c->thresh || hnext == 0.0) c->done = 1;
    else if (c->iters >= c->maxit) { c->status = 2; c->done = 1; }
    else if (j + 1 >= m) c->done = 2;   // cycle full: restart
}

__global__ __launch_bounds__(ST) void k_gm_scalar(Ctrl* c, const double* __restrict__ partials,
                                                  int nparts, int nv, int j, int op, double val) {
    __shared__ double sums[kMaxRestart + 2];
    __shared__ double red[SNW];
    __shared__ double sH[kMaxRestart + 1], sCS[kMaxRestart], sSN[kMaxRestart];
    __shared__ double sR[kMaxRestart * kMaxRestart];
    const int m = c->gm_m;
    const int oH = 0, oCS = (m + 1) * m, oSN = oCS + m, oG = oSN + m, oY = oG + m + 1, oT = oY + m;
    const int oS = oT + m + 1;
    (void)oCS;
    double* gm = c->gm;
    const int tid = threadIdx.x;
    if (op == GM_SOLVE) {
        // back substitution R y = g on the rotated Hessenberg matrix; the
        // update takes the stored basis vectors, so y_i carries s_i
        const int k = c->gm_k;
        for (int e = tid; e < k * k; e += ST) {
            const int i = e % k, l = e / k;
            if (i <= l) sR[i + kMaxRestart * l] = gm[oH + i + (m + 1) * l];
        }
        for (int i = tid; i < k; i += ST) { sH[i] = gm[oG + i]; sCS[i] = gm[oS + i]; }
        __syncthreads();
        if (tid == 0) {
            for (int i = k - 1; i >= 0; --i) {
                double s = sH[i];
                for (int l = i + 1; l < k; ++l) s -= sR[i + kMaxRestart * l] * sSN[l];
                sSN[i] = s / sR[i + kMaxRestart * i];
            }
        }
        __syncthreads();
        for (int i = tid; i < k; i += ST) gm[oY + i] = sSN[i] * sCS[i];
        return;
    }
    if (c->done) return;
    const int lane = tid & 63, wv = tid >> 6;
    // GM_H1 / GM_H2 / GM_H2S carry one more row: ||w||^2 / ||w'||^2.  GM_STEP reads
    // a norm from the partials only after a second Gram-Schmidt pass.  GM_NEXT
    // reads the single row nv.
    const int rows = (op == GM_H1 || op == GM_H2 || op == GM_H2S) ? nv + 1
                     : (op == GM_STEP && !c->gm_reorth)          ? 0
                     : op == GM_NEXT                             ? 1
                                                                 : nv;
    const double* src = op == GM_NEXT ? partials + (long)nv * nparts : partials;
    if (rows > 0 && rows <= SNW) {
        const int wpr = SNW / rows;   // wavefronts per row
        const int r = wv / wpr, q = wv - r * wpr;
        double acc = 0.0;
        if (r < rows) {
            const double* p = src + (long)r * nparts;
#pragma unroll 4
            for (int t = q * 64 + lane; t < nparts; t += wpr * 64) acc += p[t];
        }
        acc = wave_sum(acc);
        if (lane == 0) red[wv] = acc;
        __syncthreads();
        if (tid < rows) {
            double s = 0.0;
            for (int k = 0; k < wpr; ++k) s += red[tid * wpr + k];
            sums[tid] = s;
        }
    } else {
        for (int i = wv; i < rows; i += SNW) {
            double acc = 0.0;
#pragma unroll 4
            for (int t = lane; t < nparts; t += 64) acc += src[(long)i * nparts + t];
            acc = wave_sum(acc);
            if (lane == 0) sums[i] = acc;
        }
    }
    __syncthreads();
    if (op == GM_COEF) {
        // w' = (w - V_j) - sum_i c_i V_i in the stored vectors is s_j^{-1} times
        // the normalised Gram-Schmidt vector: H[i, j] = s_i s_j V_i^T (w - V_j)
        // (+1 on the diagonal), c_i = s_i^2 V_i^T (w - V_j)
        if (tid < nv) {
            const double sj = gm[oS + j], si = gm[oS + tid];
            gm[oT + tid] = si * si * sums[tid];
            gm[oH + tid + (m + 1) * j] = si * sj * sums[tid] + (tid == j ? 1.0 : 0.0);
        }
        return;
    }
    if (op == GM_NEXT) {
        // V_j = w' of column j - 1: H[j, j-1] = s_{j-1} ||V_j||, s_j = 1 / ||V_j||
        const double S = sums[0];
        if (!gm_isfinite(S)) {
            if (tid == 0) { c->status = 4; c->done = 1; }
            return;
        }
        const double nrm = sqrt(S);
        const double hnext = gm[oS + j - 1] * nrm;
        if (tid == 0) gm[oS + j] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        gm_givens(c, gm, m, j - 1, hnext, sH, sCS, sSN);
        return;
    }
    if (op == GM_H1) {
        // coefficients of the shifted pass (kept for it in the h2 slot) and
        // the Hessenberg column of P^{-1} A = (P^{-1} A - I) + I
        if (tid < nv) {
            gm[oT + tid] = sums[tid];
            gm[oH + tid + (m + 1) * j] = sums[tid] + (tid == j ? 1.0 : 0.0);
        }
        if (tid == 0) c->gm_w2 = sums[nv];
        return;
    }
    if (op == GM_H2 || op == GM_H2S) {
        // Daniel-Gragg-Kaufman-Stewart test: keep w' when the first pass
        // removed less than a fraction 1 - gm_eta2 of ||w||^2 (gm_eta2 = 0.5:
        // half); otherwise take the second pass (its coefficients h2 are
        // added to the Hessenberg column).  gm_eta2 = 0: never (the host
        // then does not launch the second pass).
        const double wp2 = sums[nv];
        const int re = c->gm_eta2 > 0.0 && !(wp2 > c->gm_eta2 * c->gm_w2);
        if (tid < nv) {
            gm[oT + tid] = re ? sums[tid] : 0.0;
            if (re) gm[oH + tid + (m + 1) * j] += sums[tid];
        }
        if (tid == 0) {
            c->gm_wp2 = wp2;
            c->gm_reorth = re;
            c->gm_rflag[j] = re;
            c->gm_nreorth += re;
        }
        if (op == GM_H2) return;
        // the combined op is only issued with a zero threshold (re = 0):
        // ||w'||^2 is the norm of the next basis vector
        if (tid == 0) gm[oT] = wp2;
        if (!gm_isfinite(wp2)) {
            if (tid == 0) { c->status = 4; c->done = 1; }
            return;
        }
        __syncthreads();
        gm_givens(c, gm, m, j, sqrt(wp2), sH, sCS, sSN);
        return;
    }
    if (op == GM_STEP) {
        const double S = c->gm_reorth ? sums[0] : c->gm_wp2;
        if (tid == 0) gm[oT] = S;
        if (!gm_isfinite(S)) {
            if (tid == 0) { c->status = 4; c->done = 1; }
            return;
        }
        gm_givens(c, gm, m, j, sqrt(S), sH, sCS, sSN);
        return;
    }
    // GM_PBB, GM_BETA: a single norm (given as val without partials)
    const double S = nparts > 0 ? sums[0] : val;
    if (op == GM_PBB) {
        if (tid == 0) {
            c->bb = S;
            c->thresh = fmax(c->tol2 * S, c->abs2);
            if (!gm_isfinite(S)) { c->status = 4; c->done = 1; }
            else if (S == 0.0) { c->rr = 0.0; c->done = 1; }
        }
    } else if (op == GM_BETA) {
        const bool go = gm_isfinite(S) && !(S <= c->thresh);
        if (tid == 0) {
            c->rr = S;
            if (!gm_isfinite(S)) { c->status = 4; c->done = 1; }
            else if (S <= c->thresh) { c->done = 1; c->gm_k = 0; }
            else {
                const double beta = sqrt(S);
                c->gm_beta = beta;
                c->gm_scale = 1.0 / beta;
                c->gm_k = 0;
                c->gm_j = 0;
            }
        }
        if (go) {
            // g = beta e1; v_0 = w / beta is stored normalised (s = 1)
            for (int i = tid; i <= m; i += ST) {
                gm[oG + i] = i == 0 ? sqrt(S) : 0.0;
                gm[oS + i] = 1.0;
            }
        }
    }
}

__global__ void k_gm_restart(Ctrl* c) {
    if (threadIdx.x == 0 && c->done == 2) c->done = 0;
}

// The vector kernels move 16 bytes per lane: lengths and strides must be
// multiples of 4 elements (true for the padded layout).
inline bool vec_ok(long N, long ld) { return N % 4 == 0 && ld % 4 == 0; }

inline int ggrid(long N) {
    long g = (N + GT * 4 - 1) / (GT * 4);
    if (g > kGmGrid) g = kGmGrid;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int gm_grid(long N) { return ggrid(N); }

// Basis sizes with a fully unrolled kernel instance (restart <= 23).
constexpr int kExactNV = 24;

#define FSD_NV_CASE(KER, T, NV, ...)                                                         \
    case NV: hipLaunchKernelGGL((KER<T, NV, true>), __VA_ARGS__); break;
#define FSD_NV_DISPATCH(KER, T, nv, ...)                                                     \
    do {                                                                                     \
        switch (nv) {                                                                        \
        FSD_NV_CASE(KER, T, 1, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 2, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 3, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 4, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 5, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 6, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 7, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 8, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 9, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 10, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 11, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 12, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 13, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 14, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 15, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 16, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 17, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 18, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 19, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 20, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 21, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 22, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 23, __VA_ARGS__)                                                 \
        FSD_NV_CASE(KER, T, 24, __VA_ARGS__)                                                 \
        default: hipLaunchKernelGGL((KER<T, kMaxRestart + 1, false>), __VA_ARGS__);          \
        }                                                                                    \
    } while (0)
static_assert(kExactNV == 24, "FSD_NV_DISPATCH lists the exact cases 1..24");

template <typename T>
hipError_t gm_mdot(const T* V, long ld, int nv, const T* w, long N, double* partials,
                   const Ctrl* ctrl, int* nparts, hipStream_t s) {
    if (!vec_ok(N, ld)) return hipErrorInvalidValue;
    const int g = ggrid(N);
    *nparts = g;
    FSD_NV_DISPATCH(k_mdot, T, nv, dim3(g), dim3(GT), 0, s, V, ld, nv, w, N, partials, ctrl);
    return hipGetLastError();
}

template <typename T>
hipError_t gm_maxpy(const T* V, long ld, int nv, const T* in, T* out, long N, const Ctrl* ctrl,
                    int hoff, int mode, double* partials, int* nparts, hipStream_t s) {
    if (!vec_ok(N, ld)) return hipErrorInvalidValue;
    const int g = ggrid(N);
    *nparts = g;
    FSD_NV_DISPATCH(k_maxpy, T, nv, dim3(g), dim3(GT), 0, s, V, ld, nv, in, out, N, ctrl, hoff,
                    mode, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t gm_update(T* x, const T* V, long ld, long N, int kmax, const Ctrl* ctrl, int yoff,
                     hipStream_t s, bool overwrite) {
    if (!vec_ok(N, ld)) return hipErrorInvalidValue;
    const int g = ggrid(N);
    FSD_NV_DISPATCH(k_gm_update, T, kmax, dim3(g), dim3(GT), 0, s, x, V, ld, N, ctrl, yoff,
                    overwrite ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t gm_scale(const T* in, T* out, long N, const Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL((k_scale<T>), dim3(ggrid(N)), dim3(GT), 0, s, in, out, N, ctrl);
    return hipGetLastError();
}

hipError_t gm_scalar(Ctrl* c, const double* partials, int nparts, int nv, int j, int op,
                     hipStream_t s, double val) {
    hipLaunchKernelGGL(k_gm_scalar, dim3(1), dim3(ST), 0, s, c, partials, nparts, nv, j, op, val);
    return hipGetLastError();
}

hipError_t gm_restart(Ctrl* c, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_restart, dim3(1), dim3(64), 0, s, c);
    return hipGetLastError();
}

#define FSD_GM_INST(T)                                                                          \
    template hipError_t gm_mdot<T>(const T*, long, int, const T*, long, double*, const Ctrl*,   \
                                   int*, hipStream_t);                                          \
    template hipError_t gm_maxpy<T>(const T*, long, int, const T*, T*, long, const Ctrl*, int,  \
                                    int, double*, int*, hipStream_t);                           \
    template hipError_t gm_update<T>(T*, const T*, long, long, int, const Ctrl*, int,           \
                                     hipStream_t, bool);                                        \
    template hipError_t gm_scale<T>(const T*, T*, long, const Ctrl*, hipStream_t);

FSD_GM_INST(double)
FSD_GM_INST(float)

}  // namespace fsd
