// Wave-resident line FFT engine for gfx950 (transform lengths L = 64..512).
//
// A group of G = L/8 lanes owns one complex line; lane tl of the group holds
// the eight points tl + G q (q = 0..7) in registers.  Every Stockham stage
// (radix 8, or 4 / 2 for the last one) works on registers: with that layout
// the inputs of butterfly b = tl + G u are registers u + r (8/R), and the
// last stage leaves the result in the same natural layout, so a forward FFT,
// a pointwise spectrum multiply and a second forward FFT chain without any
// data movement.  Between stages the group exchanges its line through a
// private LDS region with wavefront-scope barriers only (the group never
// spans two wavefronts), so workgroup barriers are needed only where a tile
// is transposed between global rows and lines.
//
// Lines per wavefront: LW = 64/G; each lane may carry LPL lines at once
// (by default LPL = 2 for float to give the float kernels the register
// reuse of the double ones; the kernels take LPL as a template parameter,
// and LPL = 1 for float is the engine with twice as many wavefronts per
// line count, for grids too small to fill the chip).
#pragma once

#include "fsd_lines.hpp"

namespace fsd {

// Wavefront-scope barrier with LDS ordering (release / acquire at
// wavefront scope around the s_barrier-free wave barrier).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lambda^{-1} or, for the two-sided system, Lambda^{-1/2}
template <typename T>
__device__ inline T lam_inv(T lam, int half) { return half ? fast_rsqrt(lam) : fast_rcp(lam); }

template <typename T, int L>
struct WGeo {
    static constexpr int G = L / 8;                  // lanes per line
    static constexpr int LW = 64 / G;                // lines per wavefront
    static constexpr int SH = sizeof(T) == 8 ? 4 : 5;
    static constexpr int LP = L + (L >> SH) + 1;     // LDS pitch of one line
    static constexpr int LPL = sizeof(T) == 8 ? 1 : 2;
    __device__ static constexpr int idx(int e) { return e + (e >> SH); }
};

// Radix-R DFT on the registers u, u + 8/R, ..., u + (R-1) 8/R.
template <int R, typename T>
__device__ inline void dft_sub(T (&xr)[8], T (&xi)[8], int u) {
    constexpr int S = 8 / R;
    T ar[R], ai[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { ar[r] = xr[u + r * S]; ai[r] = xi[u + r * S]; }
    dft<R>(ar, ai);
#pragma unroll
    for (int r = 0; r < R; ++r) { xr[u + r * S] = ar[r]; xi[u + r * S] = ai[r]; }
}

// Twiddles of every stage after the first, computed once per kernel into
// registers.  Stage s (radix R, span M) needs (R-1)(8/R) values per lane:
// w^{r k} with w = exp(-2 pi i/(M R)), k = (tl + G u) mod M.
template <int L>
struct TwPlan {
    static constexpr Plan P = make_plan(L);
    static constexpr int count(int upto) {
        int c = 0, M = 1;
        for (int s = 0; s < upto && s < P.nst; ++s) {
            if (s > 0) c += (P.r[s] - 1) * (8 / P.r[s]);
            M *= P.r[s];
        }
        return c;
    }
    static constexpr int span(int s) {
        int M = 1;
        for (int t = 0; t < s; ++t) M *= P.r[t];
        return M;
    }
    static constexpr int NTW = count(8) > 0 ? count(8) : 1;
};

template <typename T, int L, int S>
__device__ inline void tw_fill(T* twr, T* twi, int tl, const T* __restrict__ tw) {
    using TP = TwPlan<L>;
    if constexpr (S < TP::P.nst) {
        constexpr int R = TP::P.r[S], M = TP::span(S), G = L / 8, SB = 8 / R;
        constexpr int OFF = TP::count(S), TWS = L / (M * R);
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int k = (tl + G * u) % M;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int t = r * k * TWS;
                twr[OFF + u * (R - 1) + r - 1] = tw[2 * t];
                twi[OFF + u * (R - 1) + r - 1] = tw[2 * t + 1];
            }
        }
        tw_fill<T, L, S + 1>(twr, twi, tl, tw);
    }
}

// float keeps the twiddles of all stages in registers (loaded once per
// kernel, reused by every FFT of the kernel); double reads them from the
// L1-resident table at the point of use, which keeps the double passes
// within 128 VGPRs.
template <typename T, int L, bool REG = (sizeof(T) == 4)>
struct Twiddles {
    T r[TwPlan<L>::NTW], i[TwPlan<L>::NTW];
    __device__ inline void load(int tl, const T* __restrict__ tw) { tw_fill<T, L, 1>(r, i, tl, tw); }
    template <int S, int R, int M>
    __device__ inline void get(int u, int rr, T& wr, T& wi) const {
        constexpr int OFF = TwPlan<L>::count(S);
        wr = r[OFF + u * (R - 1) + rr - 1];
        wi = i[OFF + u * (R - 1) + rr - 1];
    }
};

template <typename T, int L>
struct Twiddles<T, L, false> {
    const T* tab;
    int tl;
    __device__ inline void load(int tl_, const T* __restrict__ tw) { tab = tw; tl = tl_; }
    template <int S, int R, int M>
    __device__ inline void get(int u, int rr, T& wr, T& wi) const {
        constexpr int G = L / 8, TWS = L / (M * R);
        const int k = (tl + G * u) % M;
        const int t = rr * k * TWS;
        wr = tab[2 * t];
        wi = tab[2 * t + 1];
    }
};

// Radix-8 DFT on registers 0..7 (even/odd split into two radix-4 DFTs).
// ZIN: inputs 4..7 are zero, so each radix-4 half reduces to one add/sub
// pair.  ZOUT: outputs 4..7 are not needed and are left unchanged.
template <typename T, bool ZIN, bool ZOUT>
__device__ inline void dft8_pruned(T (&xr)[8], T (&xi)[8]) {
    const T r2 = T(0.70710678118654752440084436210485);
    T er[4], ei[4], orr[4], oi[4];
    if constexpr (ZIN) {
        // even half {x0, x2, 0, 0}, odd half {x1, x3, 0, 0}
        er[0] = xr[0] + xr[2]; ei[0] = xi[0] + xi[2];
        er[2] = xr[0] - xr[2]; ei[2] = xi[0] - xi[2];
        er[1] = xr[0] + xi[2]; ei[1] = xi[0] - xr[2];
        er[3] = xr[0] - xi[2]; ei[3] = xi[0] + xr[2];
        orr[0] = xr[1] + xr[3]; oi[0] = xi[1] + xi[3];
        orr[2] = xr[1] - xr[3]; oi[2] = xi[1] - xi[3];
        orr[1] = xr[1] + xi[3]; oi[1] = xi[1] - xr[3];
        orr[3] = xr[1] - xi[3]; oi[3] = xi[1] + xr[3];
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            er[j] = xr[2 * j];      ei[j] = xi[2 * j];
            orr[j] = xr[2 * j + 1]; oi[j] = xi[2 * j + 1];
        }
        dft4(er, ei);
        dft4(orr, oi);
    }
    // odd half scaled by w8^s, s = 0..3: 1, (1-i)/sqrt2, -i, -(1+i)/sqrt2
    const T w1r = r2 * (orr[1] + oi[1]), w1i = r2 * (oi[1] - orr[1]);
    const T w2r = oi[2], w2i = -orr[2];
    const T w3r = r2 * (oi[3] - orr[3]), w3i = -r2 * (orr[3] + oi[3]);
    const T wr[4] = {orr[0], w1r, w2r, w3r}, wi[4] = {oi[0], w1i, w2i, w3i};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        xr[s] = er[s] + wr[s];
        xi[s] = ei[s] + wi[s];
        if constexpr (!ZOUT) {
            xr[s + 4] = er[s] - wr[s];
            xi[s + 4] = ei[s] - wi[s];
        }
    }
}

// One stage (radix R, span M) on the registers of lane tl.  ZIN: registers
// 4..7 hold zeros (first stage of a zero-padded line; radix 8 only), so the
// radix-8 DFT skips them.  ZOUT: only outputs 0..3 are needed (last stage,
// radix 8).
template <typename T, int L, int R, int M, int S, bool ZIN, bool ZOUT>
__device__ inline void wstage(T (&xr)[8], T (&xi)[8], const Twiddles<T, L>& tw) {
    constexpr int SB = 8 / R;
#pragma unroll
    for (int u = 0; u < SB; ++u) {
        if constexpr (M > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                T wr, wi;
                tw.template get<S, R, M>(u, r, wr, wi);
                const int q = u + r * SB;
                const T a = xr[q], b = xi[q];
                xr[q] = a * wr - b * wi;
                xi[q] = a * wi + b * wr;
            }
        }
        if constexpr (R == 8 && (ZIN || ZOUT)) {
            dft8_pruned<T, ZIN, ZOUT>(xr, xi);
        } else {
            dft_sub<R, T>(xr, xi, u);
        }
    }
}

// Exchange after a non-final stage (radix R, span M): scatter the outputs
// Y[(b/M) M R + b%M + s M] to the line region, read back X[tl + G q].
template <typename T, int L, int R, int M>
__device__ inline void wexchange(T (&xr)[8], T (&xi)[8], int tl, T* re, T* im) {
    using W = WGeo<T, L>;
    constexpr int G = W::G, S = 8 / R;
#pragma unroll
    for (int u = 0; u < S; ++u) {
        const int b = tl + G * u;
        const int base = (b / M) * M * R + b % M;
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int e = W::idx(base + s * M);
            re[e] = xr[u + s * S];
            im[e] = xi[u + s * S];
        }
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = W::idx(tl + G * q);
        xr[q] = re[e];
        xi[q] = im[e];
    }
    wave_sync();
}

template <typename T, int L, int S, int M, bool ZIN, bool ZOUT>
struct WRun {
    __device__ static inline void run(T (&xr)[8], T (&xi)[8], int tl, const Twiddles<T, L>& tw,
                                      T* re, T* im) {
        constexpr Plan P = make_plan(L);
        if constexpr (S < P.nst) {
            constexpr int R = P.r[S];
            constexpr bool zin = ZIN && S == 0 && R == 8;
            constexpr bool zout = ZOUT && S + 1 == P.nst && R == 8;
            wstage<T, L, R, M, S, zin, zout>(xr, xi, tw);
            if constexpr (S + 1 < P.nst) wexchange<T, L, R, M>(xr, xi, tl, re, im);
            WRun<T, L, S + 1, M * R, ZIN, ZOUT>::run(xr, xi, tl, tw, re, im);
        }
    }
};

// Forward FFT of one line held as points tl + G q; LDS region re/im of
// length WGeo::LP is private to the lane group.  ZIN: points q >= 4 are zero
// (zero-padded input); ZOUT: only points q < 4 of the result are used.
template <typename T, int L, bool ZIN = false, bool ZOUT = false>
__device__ inline void wfft(T (&xr)[8], T (&xi)[8], int tl, const Twiddles<T, L>& tw, T* re, T* im) {
    WRun<T, L, 0, 1, ZIN, ZOUT>::run(xr, xi, tl, tw, re, im);
}

// NL lines of one lane group in lock-step: every stage runs on all NL lines,
// and each exchange writes all of them before one wavefront barrier and
// reads them back before the next, so the LDS round trips of the lines
// overlap (one barrier pair per stage instead of NL).
template <typename T, int L, int R, int M, int NL>
__device__ inline void wexchange_n(T (&xr)[NL][8], T (&xi)[NL][8], int tl, T* const (&re)[NL],
                                   T* const (&im)[NL]) {
    using W = WGeo<T, L>;
    constexpr int G = W::G, S = 8 / R;
#pragma unroll
    for (int p = 0; p < NL; ++p) {
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int b = tl + G * u;
            const int base = (b / M) * M * R + b % M;
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int e = W::idx(base + s * M);
                re[p][e] = xr[p][u + s * S];
                im[p][e] = xi[p][u + s * S];
            }
        }
    }
    wave_sync();
#pragma unroll
    for (int p = 0; p < NL; ++p) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = W::idx(tl + G * q);
            xr[p][q] = re[p][e];
            xi[p][q] = im[p][e];
        }
    }
    wave_sync();
}

template <typename T, int L, int S, int M, bool ZIN, bool ZOUT, int NL>
struct WRunN {
    __device__ static inline void run(T (&xr)[NL][8], T (&xi)[NL][8], int tl,
                                      const Twiddles<T, L>& tw, T* const (&re)[NL],
                                      T* const (&im)[NL]) {
        constexpr Plan P = make_plan(L);
        if constexpr (S < P.nst) {
            constexpr int R = P.r[S];
            constexpr bool zin = ZIN && S == 0 && R == 8;
            constexpr bool zout = ZOUT && S + 1 == P.nst && R == 8;
#pragma unroll
            for (int p = 0; p < NL; ++p) wstage<T, L, R, M, S, zin, zout>(xr[p], xi[p], tw);
            if constexpr (S + 1 < P.nst) wexchange_n<T, L, R, M, NL>(xr, xi, tl, re, im);
            WRunN<T, L, S + 1, M * R, ZIN, ZOUT, NL>::run(xr, xi, tl, tw, re, im);
        }
    }
};

// Forward FFTs of NL lines (line p in xr[p], xi[p], LDS region re[p], im[p]).
template <typename T, int L, bool ZIN, bool ZOUT, int NL>
__device__ inline void wfft_n(T (&xr)[NL][8], T (&xi)[NL][8], int tl, const Twiddles<T, L>& tw,
                              T* const (&re)[NL], T* const (&im)[NL]) {
    WRunN<T, L, 0, 1, ZIN, ZOUT, NL>::run(xr, xi, tl, tw, re, im);
}

// Toeplitz spectrum multiply in registers: Y = conj(C Z).
template <typename T, int L>
__device__ inline void wspec(T (&xr)[8], T (&xi)[8], int tl, const T* __restrict__ spec) {
    constexpr int G = L / 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int f = tl + G * q;
        const T cr = spec[2 * f], ci = spec[2 * f + 1];
        const T zr = xr[q], zi = xi[q];
        xr[q] = cr * zr - ci * zi;
        xi[q] = -(cr * zi + ci * zr);
    }
}

// The same product with the spectrum values already in registers.
template <typename T>
__device__ inline void wspec_regs(T (&xr)[8], T (&xi)[8], const T (&cr)[8], const T (&ci)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const T zr = xr[q], zi = xi[q];
        xr[q] = cr[q] * zr - ci[q] * zi;
        xi[q] = -(cr[q] * zi + ci[q] * zr);
    }
}

template <int L>
constexpr bool wave_engine_length() {
    return L == 64 || L == 128 || L == 256 || L == 512;
}

// ------------------------------------------------------------ x-axis pass
// Workgroup: 4 wavefronts; each lane group handles LPL complex lines
// (2 LPL rows).  No workgroup barrier: loads and stores go straight between
// global rows and registers.

template <typename T, int L, int LPLV = WGeo<T, L>::LPL>
struct WX {
    using W = WGeo<T, L>;
    static constexpr int NW = 4;
    static constexpr int NT = 64 * NW;
    static constexpr int LINES = NW * W::LW * LPLV;   // complex lines per workgroup
};

// The prologue (PRO_*) is a template parameter: one lean kernel per mode.
// Float is held to four wavefronts per SIMD (128 VGPRs): the LDS of a
// workgroup allows four, and the two-line float kernel would take a few
// registers more than that budget.
template <typename T, int L, int PRO, int LPLV = WGeo<T, L>::LPL>
__global__ __launch_bounds__(256) void k2_toep_x(ToepArgs<T> a) {
    using W = WGeo<T, L>;
    constexpr int G = W::G, LW = W::LW, LPL = LPLV, LP = W::LP;
    constexpr int NN = L / 2 - 1;   // line length n; points q >= 4 are the zero padding
    if (a.ctrl && a.ctrl->done) return;
    __shared__ T s_re[WX<T, L, LPLV>::LINES * LP];
    __shared__ T s_im[WX<T, L, LPLV>::LINES * LP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / G, tl = lane % G;
    const int P1 = a.g.P1, nrows = a.g.nrows;
    T beta = 0, scale = 1;
    bool first = true;
    if constexpr (PRO == PRO_PUPDATE) { first = a.ctrl->first != 0; beta = (T)a.ctrl->beta; }
    if constexpr (PRO == PRO_SCALE) scale = (T)a.ctrl->gm_scale;

    T xr[LPL][8], xi[LPL][8];
    T* re[LPL];
    T* im[LPL];
    // Every load of the lane is issued before the prologue's first store:
    // pro_p may alias u_fft as far as the compiler knows, so a store between
    // two loads would make each load wait for the one before it.
    T pv[PRO == PRO_PUPDATE ? LPL : 1][2][4];   // PRO_PUPDATE: the old p
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        const int slot = wave * LW * LPL + g + LW * p;
        re[p] = s_re + slot * LP;
        im[p] = s_im + slot * LP;
        const int line = blockIdx.x * WX<T, L, LPLV>::LINES + slot;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = 2 * line + h;
            const bool rv = row < nrows;
            const long base = (long)row * P1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = tl + G * q;
                T z = 0;
                if (rv && e < NN) {
                    z = a.u_fft[base + e];
                    if constexpr (PRO == PRO_PUPDATE) pv[p][h][q] = first ? T(0) : a.pro_p[base + e];
                } else if constexpr (PRO == PRO_PUPDATE) {
                    pv[p][h][q] = T(0);
                }
                if (h == 0) xr[p][q] = z; else xi[p][q] = z;
            }
        }
#pragma unroll
        for (int q = 4; q < 8; ++q) { xr[p][q] = T(0); xi[p][q] = T(0); }
    }
    if constexpr (PRO == PRO_ARNOLDI) {
        // Gram-Schmidt update of the GMRES basis in the prologue: first
        // u_in - V_{nv-1} (exact where the two agree to a factor of 2: the
        // preconditioned operator is close to the identity), then the
        // projections c_i V_i, the loads of two basis vectors in flight at a time
        const int nv = a.gs_nv;
        const T* __restrict__ V = a.gs_V;
        const long ld = a.gs_ld;
        const double* cg = a.ctrl->gm + a.gs_hoff;
        auto load_rows = [&](const T* __restrict__ src, T (&t)[LPL][2][4]) {
#pragma unroll
            for (int p = 0; p < LPL; ++p) {
                const int line = blockIdx.x * WX<T, L, LPLV>::LINES + wave * LW * LPL + g + LW * p;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int row = 2 * line + h;
                    const bool rv = row < nrows;
                    const long base = (long)row * P1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int e = tl + G * q;
                        t[p][h][q] = (rv && e < NN) ? src[base + e] : T(0);
                    }
                }
            }
        };
        auto sub = [&](const T (&t)[LPL][2][4], T c) {
#pragma unroll
            for (int p = 0; p < LPL; ++p) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    xr[p][q] -= c * t[p][0][q];
                    xi[p][q] -= c * t[p][1][q];
                }
            }
        };
        T t0[LPL][2][4], t1[LPL][2][4];
        load_rows(V + (long)(nv - 1) * ld, t0);
        sub(t0, T(1));
        int i = 0;
        for (; i + 2 <= nv; i += 2) {
            load_rows(V + (long)i * ld, t0);
            load_rows(V + (long)(i + 1) * ld, t1);
            sub(t0, (T)cg[i]);
            sub(t1, (T)cg[i + 1]);
        }
        if (i < nv) {
            load_rows(V + (long)i * ld, t0);
            sub(t0, (T)cg[i]);
        }
        double nacc = 0.0;
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
            const int line = blockIdx.x * WX<T, L, LPLV>::LINES + wave * LW * LPL + g + LW * p;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = 2 * line + h;
                const bool rv = row < nrows;
                const long base = (long)row * P1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = tl + G * q;
                    const T v = h == 0 ? xr[p][q] : xi[p][q];
                    if (rv && e < NN) {
                        st_nt(a.pro_p + base + e, v);
                        nacc += (double)v * (double)v;
                    }
                }
            }
        }
        __shared__ double s_nrm[WX<T, L, LPLV>::NW];
        const double bs = block_sum<WX<T, L, LPLV>::NT>(nacc, s_nrm);
        if (threadIdx.x == 0) a.partials[blockIdx.x] = bs;
    }
    if constexpr (PRO == PRO_PUPDATE || PRO == PRO_SCALE) {
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
            const int line = blockIdx.x * WX<T, L, LPLV>::LINES + wave * LW * LPL + g + LW * p;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = 2 * line + h;
                const bool rv = row < nrows;
                const long base = (long)row * P1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = tl + G * q;
                    T& v = h == 0 ? xr[p][q] : xi[p][q];
                    if constexpr (PRO == PRO_PUPDATE) {
                        if (!first) v += beta * pv[p][h][q];
                    } else {
                        v *= scale;
                    }
                    if (rv && e < NN) st_nt(a.pro_p + base + e, v);
                }
            }
        }
    }
    if (a.o2) {
        // A_n u along x from natural-order copies of the lines (points 0..n)
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = W::idx(tl + G * q);
                re[p][e] = xr[p][q];
                im[p][e] = xi[p][q];
            }
        }
        wave_sync();
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
            const int line = blockIdx.x * WX<T, L, LPLV>::LINES + wave * LW * LPL + g + LW * p;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = 2 * line + h;
                if (row >= nrows) break;
                const T* src = h ? im[p] : re[p];
                const long base = (long)row * P1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = tl + G * q;
                    if (e < NN) {
                        const T l = e > 0 ? src[W::idx(e - 1)] : T(0);
                        const T r = src[W::idx(e + 1)];
                        const T c = h ? xi[p][q] : xr[p][q];
                        st_nt(a.o2 + base + e, (l + T(6) * c + r) * T(0.125));
                    }
                }
            }
        }
        wave_sync();
    }
    Twiddles<T, L> tw;
    tw.load(tl, a.tw);
    // float: the spectrum at this lane's frequencies is loaded before the
    // forward transform (the register budget allows it at this occupancy),
    // so its latency overlaps the transform
    T cr[8], ci[8];
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int f = tl + G * q;
            cr[q] = a.spec[2 * f];
            ci[q] = a.spec[2 * f + 1];
        }
    }
    wfft_n<T, L, true, false, LPL>(xr, xi, tl, tw, re, im);
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        if constexpr (sizeof(T) == 4) wspec_regs<T>(xr[p], xi[p], cr, ci);
        else wspec<T, L>(xr[p], xi[p], tl, a.spec);
    }
    wfft_n<T, L, false, true, LPL>(xr, xi, tl, tw, re, im);
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        const int line = blockIdx.x * WX<T, L, LPLV>::LINES + wave * LW * LPL + g + LW * p;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = 2 * line + h;
            if (row >= nrows) break;
            const long base = (long)row * P1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = tl + G * q;
                if (e < NN) st_nt(a.o1 + base + e, h ? -xi[p][q] : xr[p][q]);
            }
        }
    }
}

// DST-I of two real lines per complex line, x axis.  Each element of a row
// is read from global memory once (points 0..L/2-1 of the odd extension);
// the mirrored half V[L-j] = -V[j] comes back through the line's LDS region
// (reading it a second time from global memory, in reversed lane order,
// measured 1.7x slower).
template <typename T, int L, int LPLV = WGeo<T, L>::LPL>
__global__ __launch_bounds__(256) void k2_dst_x(DstArgs<T> a) {
    using W = WGeo<T, L>;
    constexpr int G = W::G, LW = W::LW, LPL = LPLV, LP = W::LP;
    constexpr int NN = L / 2 - 1;
    if (a.ctrl && a.ctrl->done) return;
    __shared__ T s_re[WX<T, L, LPLV>::LINES * LP];
    __shared__ T s_im[WX<T, L, LPLV>::LINES * LP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / G, tl = lane % G;
    // the twiddles (float: registers, loaded from global memory) are
    // requested before the line loads, so both arrive in one wait (measured
    // faster for this pass only: 35.8 -> 34.4 us at 255^3)
    Twiddles<T, L> tw;
    tw.load(tl, a.tw);
    const int P1 = a.g.P1, nrows = a.g.nrows;
    T xr[LPL][8], xi[LPL][8];
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        const int line = blockIdx.x * WX<T, L, LPLV>::LINES + wave * LW * LPL + g + LW * p;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = 2 * line + h;
            const bool rv = row < nrows;
            const long base = (long)row * P1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // odd extension: V[0] = V[n+1] = 0, V[j] = u[j-1] (j = 1..n)
                const int e = tl + G * q;
                const T v = (rv && e >= 1) ? a.u[base + e - 1] : T(0);
                if (h == 0) xr[p][q] = v; else xi[p][q] = v;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        const int slot = wave * LW * LPL + g + LW * p;
        T* re = s_re + slot * LP;
        T* im = s_im + slot * LP;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = W::idx(tl + G * q);
            re[e] = xr[p][q];
            im[e] = xi[p][q];
        }
        if (tl == 0) { re[W::idx(NN + 1)] = T(0); im[W::idx(NN + 1)] = T(0); }
    }
    wave_sync();
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        const int slot = wave * LW * LPL + g + LW * p;
        const T* re = s_re + slot * LP;
        const T* im = s_im + slot * LP;
#pragma unroll
        for (int q = 4; q < 8; ++q) {
            const int e = tl + G * q;   // V[e] = -V[L - e], L - e in 1..n+1
            xr[p][q] = -re[W::idx(L - e)];
            xi[p][q] = -im[W::idx(L - e)];
        }
    }
    wave_sync();
    {
        T* re[LPL];
        T* im[LPL];
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
            const int slot = wave * LW * LPL + g + LW * p;
            re[p] = s_re + slot * LP;
            im[p] = s_im + slot * LP;
        }
        wfft_n<T, L, false, true, LPL>(xr, xi, tl, tw, re, im);
    }
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        const int line = blockIdx.x * WX<T, L, LPLV>::LINES + wave * LW * LPL + g + LW * p;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = 2 * line + h;
            if (row >= nrows) break;
            const long base = (long)row * P1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = tl + G * q;   // DST index k = 1..n -> output k-1
                if (k >= 1) st_nt(a.o + base + k - 1, h ? xr[p][q] * a.c : -xi[p][q] * a.c);
            }
        }
    }
}

// n = L/2 - 1 for every pass (L = 2(n + 1)), so the per-thread trip
// counts are constants: all loads of a thread are issued before the first
// LDS store (one memory latency per tile instead of one per element).
// Only points 0..L/2 of the odd extension are staged (V[0] = V[n+1] = 0,
// V[j] = u[j-1]); the lane groups read the mirrored half V[L-j] = -V[j]
// from there (line_regs_odd).
template <typename T, int L, int GRP>
__device__ inline void dst_load_strided_w(const T* __restrict__ u, T* line, long base, long es,
                                          int ig) {
    using W = WGeo<T, L>;
    constexpr int NN = L / 2 - 1, NIT = (NN + GRP - 1) / GRP;
    T v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = ig + it * GRP;
        v[it] = i < NN ? u[base + (long)i * es] : T(0);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = ig + it * GRP;
        if (i < NN) line[W::idx(i + 1)] = v[it];
    }
    if (ig == 0) { line[W::idx(0)] = 0; line[W::idx(NN + 1)] = 0; }
}

// Registers of one complex line (points tl + G q) from a line region that
// holds points 0..L/2 of two odd extensions (re, im).
template <typename T, int L>
__device__ inline void line_regs_odd(T (&xr)[8], T (&xi)[8], int tl, const T* re, const T* im) {
    using W = WGeo<T, L>;
    constexpr int G = W::G;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = W::idx(tl + G * q);
        xr[q] = re[e];
        xi[q] = im[e];
    }
#pragma unroll
    for (int q = 4; q < 8; ++q) {
        const int e = W::idx(L - tl - G * q);   // L - e in 1..L/2
        xr[q] = -re[e];
        xi[q] = -im[e];
    }
}

// Double strided passes of length >= 256 keep the twiddle table (L complex
// values) in LDS when it fits beside the tile within half the LDS of a CU
// (two workgroups per CU): the stages then read their twiddles there
// instead of waiting on the cache.  The table is loaded with the tile's
// rows (one wait).
template <typename T, int L>
struct TwLds {
    template <int BASE_BYTES>
    static constexpr bool on() {
        return sizeof(T) == 8 && L >= 256 && BASE_BYTES + 2 * L * (int)sizeof(T) <= 80 * 1024;
    }
};

template <typename T, int L, int NT, bool ON>
struct TwStager {
    static constexpr int N = ON ? 2 * L : 1, NI = ON ? (2 * L + NT - 1) / NT : 1;
    T v[NI];
    __device__ inline void load(const T* __restrict__ tw, int tid) {
        if constexpr (ON) {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int e = tid + k * NT;
                v[k] = e < 2 * L ? tw[e] : T(0);
            }
        }
    }
    __device__ inline void store(T* s_tw, int tid) const {
        if constexpr (ON) {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int e = tid + k * NT;
                if (e < 2 * L) s_tw[e] = v[k];
            }
        }
    }
};

// ------------------------------------------------------ strided y/z passes
// Tile: NCL = 8 (double) or 16 (float) complex lines = 2 NCL consecutive x
// positions (a 128-byte row segment) at one outer index.  Three workgroup
// barriers: after the row loads, after the A_n stencil, before the row stores.

template <typename T, int L, int LPLV = WGeo<T, L>::LPL>
struct WS {
    using W = WGeo<T, L>;
    static constexpr int NCL = sizeof(T) == 8 ? 8 : 16;
    static constexpr int TX = 2 * NCL;
    static constexpr int NW = NCL / (W::LW * LPLV);
    static constexpr int NT = 64 * NW;
    static constexpr int GRP = NT / TX;
    // Minimum wavefronts per SIMD the strided DST pass is compiled for:
    // float holds 128 VGPRs without spilling; the double SCALE variant does
    // not (it would spill ~100 bytes per lane, measured slower than running
    // at lower occupancy), so double takes no cap.
    static constexpr int MINW = sizeof(T) == 8 ? 1 : 4;
};

template <typename T, int L, int LPLV = WGeo<T, L>::LPL>
__global__ __launch_bounds__((WS<T, L, LPLV>::NT)) void k2_toep_s(ToepArgs<T> a) {
    using W = WGeo<T, L>;
    using S = WS<T, L, LPLV>;
    constexpr int G = W::G, LW = W::LW, LPL = LPLV, LP = W::LP;
    constexpr int NCL = S::NCL, TX = S::TX, NT = S::NT, GRP = S::GRP;
    if (a.ctrl && a.ctrl->done) return;
    constexpr bool TWL = TwLds<T, L>::template on<2 * NCL * LP * (int)sizeof(T) + NT / 8>();
    __shared__ T s_re[NCL * LP];
    __shared__ T s_im[NCL * LP];
    __shared__ T s_tw[TwStager<T, L, NT, TWL>::N];
    __shared__ double s_red[NT / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane / G, tl = lane % G;
    const int n = a.g.n, P1 = a.g.P1;
    const long es = a.g.estride;
    const int ntx = P1 / TX;
    const int xt = blockIdx.x % ntx, o = blockIdx.x / ntx;
    const int x0 = xt * TX;
    // row-transpose mapping
    const int xl = tid % TX, ig = tid / TX;
    const long base = (long)o * a.g.ostride + x0 + xl;
    T* rline = ((xl & 1) ? s_im : s_re) + (xl >> 1) * LP;
    TwStager<T, L, NT, TWL> tws;
    tws.load(a.tw, tid);
    // n = L/2 - 1 (L = 2(n + 1)): constant trip counts, loads issued first
    constexpr int NN = L / 2 - 1, NIT = (NN + GRP - 1) / GRP, NZ = (L - NN + GRP - 1) / GRP;
    {
        T v[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = ig + it * GRP;
            v[it] = i < NN ? a.u_fft[base + (long)i * es] : T(0);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = ig + it * GRP;
            if (i < NN) rline[W::idx(i)] = v[it];
        }
#pragma unroll
        for (int it = 0; it < NZ; ++it) {
            const int i = NN + ig + it * GRP;
            if (i < L) rline[W::idx(i)] = T(0);
        }
    }
    tws.store(s_tw, tid);
    __syncthreads();
    const bool pad_line = x0 + xl >= a.g.nx;
    if (a.o2) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = ig + it * GRP;
            if (i < NN) {
                const T l = i > 0 ? rline[W::idx(i - 1)] : T(0);
                const T c = rline[W::idx(i)];
                const T r = rline[W::idx(i + 1)];
                st_nt(a.o2 + base + (long)i * es, pad_line ? T(0) : (l + T(6) * c + r) * T(0.125));
            }
        }
    }
    // lane groups pull their lines
    T xr[LPL][8], xi[LPL][8];
#pragma unroll
    for (int p = 0; p < LPL; ++p) {
        const int slot = wave * LW * LPL + g + LW * p;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = W::idx(tl + G * q);
            xr[p][q] = s_re[slot * LP + e];
            xi[p][q] = s_im[slot * LP + e];
        }
    }
    __syncthreads();
    Twiddles<T, L> tw;
    tw.load(tl, TWL ? s_tw : a.tw);
    {
        T* re[LPL];
        T* im[LPL];
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
            const int slot = wave * LW * LPL + g + LW * p;
            re[p] = s_re + slot * LP;
            im[p] = s_im + slot * LP;
        }
        wfft_n<T, L, true, false, LPL>(xr, xi, tl, tw, re, im);
#pragma unroll
        for (int p = 0; p < LPL; ++p) wspec<T, L>(xr[p], xi[p], tl, a.spec);
        wfft_n<T, L, false, true, LPL>(xr, xi, tl, tw, re, im);
        // points 0..n-1 are the ones read back (outputs q < 4; ZOUT)
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = W::idx(tl + G * q);
                re[p][e] = xr[p][q];
                im[p][e] = xi[p][q];
            }
        }
    }
    __syncthreads();
    // row stores with the A_n stencil on u_sten and the epilogue; each
    // thread owns CH consecutive line points, and every global value it
    // needs (stencil neighbours, epilogue operand) is loaded before the
    // first use
    constexpr int CH = (NN + GRP - 1) / GRP;
    const int ib = ig * CH;
    const T sgn = (xl & 1) ? T(-1) : T(1);
    const int x = x0 + xl;
    double acc = 0.0;
    const bool has_sten = a.u_sten != nullptr;
    T st[CH + 2];
    T ep[CH];
#pragma unroll
    for (int k = 0; k < CH + 2; ++k) {
        const int i = ib - 1 + k;
        st[k] = (has_sten && i >= 0 && i < NN) ? a.u_sten[base + (long)i * es] : T(0);
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int i = ib + k;
        T e = 0;
        if (i < NN) {
            const long gi = base + (long)i * es;
            if (a.epi == EPI_ADD_F) {
                if (x < a.g.n1)
                    e = (T)(a.dt * a.F[x + (long)a.g.n1 * ((long)i * a.g.fr_i + (long)o * a.g.fr_o)]);
            } else if (a.epi == EPI_DOT_P) {
                e = a.dot_p[gi];
            } else if (a.epi == EPI_RESID) {
                e = a.b[gi];
            }
        }
        ep[k] = e;
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int i = ib + k;
        if (i >= NN) break;
        T v = sgn * rline[W::idx(i)];
        if (has_sten) v += (st[k] + T(6) * st[k + 1] + st[k + 2]) * T(0.125);
        const long gi = base + (long)i * es;
        if (pad_line) v = T(0);
        if (a.epi == EPI_ADD_F) {
            v += ep[k];
        } else if (a.epi == EPI_DOT_P) {
            acc += (double)ep[k] * (double)v;
        } else if (a.epi == EPI_RESID) {
            v = ep[k] - v;
            acc += (double)v * (double)v;
        }
        st_nt(a.o1 + gi, v);
    }
    if (a.epi == EPI_DOT_P || a.epi == EPI_RESID) {
        const double s = block_sum<NT>(acc, s_red);
        if (tid == 0) a.partials[blockIdx.x] = s;
    }
}

// Strided DST pass; with SCALE, the last-axis pass S Lambda^{-1} S with the
// Parseval partial sums of (r, P^{-1} r).  The tile's LDS allows about four
// wavefronts per SIMD; for float the register budget is held to that (128
// VGPRs), or the SCALE variant at L = 512 would drop to one workgroup per CU.
template <typename T, int L, bool SCALE, int LPLV = WGeo<T, L>::LPL>
__global__ __launch_bounds__((WS<T, L, LPLV>::NT))
__attribute__((amdgpu_waves_per_eu(WS<T, L, LPLV>::MINW))) void k2_dst_s(DstArgs<T> a) {
    using W = WGeo<T, L>;
    using S = WS<T, L, LPLV>;
    constexpr int G = W::G, LW = W::LW, LPL = LPLV, LP = W::LP;
    constexpr int NCL = S::NCL, TX = S::TX, NT = S::NT, GRP = S::GRP;
    if (a.ctrl && a.ctrl->done) return;
    __shared__ T s_re[NCL * LP];
    __shared__ T s_im[NCL * LP];
    __shared__ T s_P[TX], s_Q[TX];
    // SCALE: the last axis's factors a_k and lc_k (k = 1..n) in LDS
    constexpr int NH = SCALE ? L / 2 : 1, NL = (NH + NT - 1) / NT;
    __shared__ T s_al[NH], s_lc[NH];
    constexpr bool TWL = TwLds<T, L>::template on<(2 * NCL * LP + 2 * TX + 2 * NH) * (int)sizeof(T) +
                                                  NT / 8>();
    __shared__ T s_tw[TwStager<T, L, NT, TWL>::N];
    __shared__ double s_red[NT / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane / G, tl = lane % G;
    const int n = a.g.n, P1 = a.g.P1;
    const long es = a.g.estride;
    const int ntx = P1 / TX;
    const int xt = blockIdx.x % ntx, o = blockIdx.x / ntx;
    const int x0 = xt * TX;
    const int xl = tid % TX, ig = tid / TX;
    const long base = (long)o * a.g.ostride + x0 + xl;
    // The factor loads are issued before the tile's row loads and stored to
    // LDS after them, so that the workgroup waits for memory once.
    T fa1 = 0, fl1 = 0, fa2 = 0, fl2 = 0;
    T al[NL], lc[NL];
    if constexpr (SCALE) {
        const int x = x0 + tid;
        if (tid < TX && x < a.g.nx) {
            fa1 = a.a1[x];
            fl1 = a.lc1[x];
            if (a.dim == 3) {
                fa2 = a.a2[o];
                fl2 = a.lc2[o];
            }
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = tid + k * NT;
            al[k] = e < n ? a.a_last[e] : T(0);
            lc[k] = e < n ? a.lc_last[e] : T(0);
        }
    }
    TwStager<T, L, NT, TWL> tws;
    tws.load(a.tw, tid);
    T* rline = ((xl & 1) ? s_im : s_re) + (xl >> 1) * LP;
    dst_load_strided_w<T, L, GRP>(a.u, rline, base, es, ig);
    tws.store(s_tw, tid);
    if constexpr (SCALE) {
        if (tid < TX) {
            T P = 0, Q = 0;
            if (x0 + tid < a.g.nx) {
                if (a.dim == 2) {
                    P = fa1 + fl1;
                    Q = fa1;
                } else {
                    P = fa2 * (fa1 + fl1) + fl2 * fa1;
                    Q = fa2 * fa1;
                }
            }
            s_P[tid] = P;
            s_Q[tid] = Q;
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = tid + k * NT;
            if (e < NH) {
                s_al[e] = al[k];
                s_lc[e] = lc[k];
            }
        }
    }
    __syncthreads();
    Twiddles<T, L> tw;
    tw.load(tl, TWL ? s_tw : a.tw);
    double acc = 0.0;
    if constexpr (!SCALE) {
        // plain DST: the LPL lines of a lane group in lock-step
        T xr[LPL][8], xi[LPL][8];
        T* re[LPL];
        T* im[LPL];
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
            const int slot = wave * LW * LPL + g + LW * p;
            re[p] = s_re + slot * LP;
            im[p] = s_im + slot * LP;
            line_regs_odd<T, L>(xr[p], xi[p], tl, re[p], im[p]);
        }
        wave_sync();
        wfft_n<T, L, false, true, LPL>(xr, xi, tl, tw, re, im);
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = W::idx(tl + G * q);
                re[p][e] = xr[p][q];
                im[p][e] = xi[p][q];
            }
        }
    } else {
        // scale pass: one line in registers at a time (register budget); a
        // lane group's LDS region is its own, so line p + 1 stays there
        // untouched while line p is transformed
#pragma unroll
        for (int p = 0; p < LPL; ++p) {
            const int slot = wave * LW * LPL + g + LW * p;
            T* re = s_re + slot * LP;
            T* im = s_im + slot * LP;
            T xr[8], xi[8];
            line_regs_odd<T, L>(xr, xi, tl, re, im);
            wave_sync();
            wfft<T, L, false, false>(xr, xi, tl, tw, re, im);
            const T P0 = s_P[2 * slot], Q0 = s_Q[2 * slot];
            const T P1v = s_P[2 * slot + 1], Q1v = s_Q[2 * slot + 1];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int f = tl + G * q;
                const int k = f <= n ? f : L - f;
                T wr = 0, wi = 0;
                if (k >= 1 && k <= n) {
                    const T ak = s_al[k - 1], lk = s_lc[k - 1];
                    const T inv0 = P0 != T(0) ? lam_inv(ak * P0 + lk * Q0, a.half) : T(0);
                    const T inv1 = P1v != T(0) ? lam_inv(ak * P1v + lk * Q1v, a.half) : T(0);
                    const T s1 = -xi[q] * a.c;
                    const T s2 = xr[q] * a.c;
                    wr = s1 * inv0;
                    wi = s2 * inv1;
                    if (f <= n)
                        acc += (a.pnorm ? (double)wr : (double)s1) * (double)wr +
                               (a.pnorm ? (double)wi : (double)s2) * (double)wi;
                }
                xr[q] = wr;
                xi[q] = wi;
            }
            wfft<T, L, false, true>(xr, xi, tl, tw, re, im);
            // points 1..n are the ones read back (outputs q < 4; ZOUT)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = W::idx(tl + G * q);
                re[e] = xr[q];
                im[e] = xi[q];
            }
        }
    }
    __syncthreads();
    const bool odd = xl & 1;
    const T* other = (odd ? s_re : s_im) + (xl >> 1) * LP;
    const bool pad_line = x0 + xl >= a.g.nx;
    constexpr int NN = L / 2 - 1;
#pragma unroll
    for (int i = ig; i < NN; i += GRP) {
        const T z = other[W::idx(i + 1)];
        st_nt(a.o + base + (long)i * es, pad_line ? T(0) : (odd ? z * a.c : -z * a.c));
    }
    if (SCALE && a.partials) {
        const double s = block_sum<NT>(acc, s_red);
        if (tid == 0) a.partials[blockIdx.x] = s;
    }
}

}  // namespace fsd
