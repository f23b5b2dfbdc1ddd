// Per-length dispatch of the line passes: float32 strided passes of length
// 512 use the column engine (fsd_cols.hpp); lengths 64..512 otherwise use
// the wave engine (fsd_wave.hpp); the other lengths the LDS-stage engine
// (fsd_lines.hpp).  A pass set to another engine (fsd_set_engine) runs on
// it where that engine supports the length.
#pragma once

#include <type_traits>

#include "fsd_cols.hpp"
#include "fsd_wave.hpp"

namespace fsd {

template <typename T, int L>
constexpr bool column_engine_length() {
    return std::is_same<T, float>::value && L == colx::L;
}

// Stage-engine tile shapes: the default lines per tile and half of it.
template <typename T, int L>
struct StageNC {
    static constexpr int D = lines_per_block(L, sizeof(T) == 8);
    static constexpr int H = D > 1 ? D / 2 : 1;
};

template <typename T, int L, template <typename, int, int> class K, typename A>
hipError_t stage_x_launch(const A& a, int* nb, hipStream_t s, int eng) {
    using NC = StageNC<T, L>;
    if (eng == ENG_STAGE_HALF && NC::H != NC::D) {
        const int g = x_blocks<T>(L, a.g.nrows, NC::H);
        if (nb) *nb = g;
        if (g) hipLaunchKernelGGL((K<T, L, NC::H>::kernel), dim3(g), dim3(Tile<T, L, NC::H>::NT), 0, s, a);
    } else {
        const int g = x_blocks<T>(L, a.g.nrows, NC::D);
        if (nb) *nb = g;
        if (g) hipLaunchKernelGGL((K<T, L, NC::D>::kernel), dim3(g), dim3(Tile<T, L, NC::D>::NT), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T, int L, template <typename, int, int> class K, typename A>
hipError_t stage_s_launch(const A& a, int* nb, hipStream_t s, int eng) {
    using NC = StageNC<T, L>;
    if (eng == ENG_STAGE_HALF && NC::H != NC::D) {
        const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer, NC::H);
        if (nb) *nb = g;
        if (g) hipLaunchKernelGGL((K<T, L, NC::H>::kernel), dim3(g), dim3(Tile<T, L, NC::H>::NT), 0, s, a);
    } else {
        const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer, NC::D);
        if (nb) *nb = g;
        if (g) hipLaunchKernelGGL((K<T, L, NC::D>::kernel), dim3(g), dim3(Tile<T, L, NC::D>::NT), 0, s, a);
    }
    return hipGetLastError();
}

// The stage engine's last-axis scale pass by the half-length DST-I: the
// tile of NC complex lines at length L/2, the same workgroup count as the
// odd-extension kernel with NC lines.
template <typename T, int L>
hipError_t stage_dstsh_launch(const DstArgs<T>& a, int* nb, hipStream_t s, int eng) {
    using NC = StageNC<T, L>;
    if (eng == ENG_STAGE_HALF && NC::H != NC::D) {
        const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer, NC::H);
        if (nb) *nb = g;
        if (g) hipLaunchKernelGGL((k_dstsh_s<T, L, NC::H>), dim3(g),
                                  dim3(Tile<T, L / 2, NC::H, dstsh_nto<T, L, NC::H>()>::NT), 0, s, a);
    } else {
        const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer, NC::D);
        if (nb) *nb = g;
        if (g) hipLaunchKernelGGL((k_dstsh_s<T, L, NC::D>), dim3(g),
                                  dim3(Tile<T, L / 2, NC::D, dstsh_nto<T, L, NC::D>()>::NT), 0, s, a);
    }
    return hipGetLastError();
}

// kernel handles of the stage engine, by tile shape
template <typename T, int L, int NC> struct KToepX { static constexpr auto kernel = k_toep_x<T, L, NC>; };
template <typename T, int L, int NC> struct KToepS { static constexpr auto kernel = k_toep_s<T, L, NC>; };
template <typename T, int L, int NC> struct KDstX { static constexpr auto kernel = k_dst_x<T, L, NC>; };
template <typename T, int L, int NC> struct KDstS { static constexpr auto kernel = k_dst_s<T, L, NC>; };
template <typename T, int L, int NC> struct KDstsS { static constexpr auto kernel = k_dsts_s<T, L, NC>; };

inline bool stage_engine(int eng) { return eng == ENG_STAGE || eng == ENG_STAGE_HALF; }

// Lines per lane group of the wave engine: the default, or one for the
// float passes on ENG_WAVE1.
template <typename T, int L>
constexpr int wave_lpl_default() { return WGeo<T, L>::LPL; }
template <typename T>
inline bool wave1(int eng) { return std::is_same<T, float>::value && eng == ENG_WAVE1; }

template <typename T, int L, int LPLV>
hipError_t wave_toep_x(const ToepArgs<T>& a, int* nb, hipStream_t s) {
    constexpr int rows = 2 * WX<T, L, LPLV>::LINES;
    constexpr int NT = WX<T, L, LPLV>::NT;
    const int g = (a.g.nrows + rows - 1) / rows;
    if (nb) *nb = g;
    if (!g) return hipSuccess;
    switch (a.pro) {
        case PRO_PUPDATE:
            hipLaunchKernelGGL((k2_toep_x<T, L, PRO_PUPDATE, LPLV>), dim3(g), dim3(NT), 0, s, a);
            break;
        case PRO_SCALE:
            hipLaunchKernelGGL((k2_toep_x<T, L, PRO_SCALE, LPLV>), dim3(g), dim3(NT), 0, s, a);
            break;
        case PRO_ARNOLDI:
            if (!a.ctrl || !a.gs_V || !a.partials || a.gs_nv < 1) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k2_toep_x<T, L, PRO_ARNOLDI, LPLV>), dim3(g), dim3(NT), 0, s, a);
            break;
        default:
            hipLaunchKernelGGL((k2_toep_x<T, L, PRO_NONE, LPLV>), dim3(g), dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T, int L, int LPLV>
hipError_t wave_dst_x(const DstArgs<T>& a, int* nb, hipStream_t s) {
    constexpr int rows = 2 * WX<T, L, LPLV>::LINES;
    const int g = (a.g.nrows + rows - 1) / rows;
    if (nb) *nb = g;
    if (g) hipLaunchKernelGGL((k2_dst_x<T, L, LPLV>), dim3(g), dim3(WX<T, L, LPLV>::NT), 0, s, a);
    return hipGetLastError();
}

template <typename T, int L, int LPLV>
hipError_t wave_toep_s(const ToepArgs<T>& a, int* nb, hipStream_t s) {
    static_assert(WS<T, L, LPLV>::TX == 2 * lines_per_block(L, sizeof(T) == 8), "tile width");
    const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer);
    if (nb) *nb = g;
    if (g) hipLaunchKernelGGL((k2_toep_s<T, L, LPLV>), dim3(g), dim3(WS<T, L, LPLV>::NT), 0, s, a);
    return hipGetLastError();
}

template <typename T, int L, bool SCALE, int LPLV>
hipError_t wave_dst_s(const DstArgs<T>& a, int* nb, hipStream_t s) {
    static_assert(WS<T, L, LPLV>::TX == 2 * lines_per_block(L, sizeof(T) == 8), "tile width");
    const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer);
    if (nb) *nb = g;
    if (g)
        hipLaunchKernelGGL((k2_dst_s<T, L, SCALE, LPLV>), dim3(g), dim3(WS<T, L, LPLV>::NT), 0, s, a);
    return hipGetLastError();
}

template <typename T, int L>
hipError_t toep_x_one(const ToepArgs<T>& a, int* nb, hipStream_t s, int eng) {
    if (a.g.n != L / 2 - 1) return hipErrorInvalidValue;   // the kernels take n = L/2 - 1
    if constexpr (wave_engine_length<L>()) {
        if (!stage_engine(eng)) {
            if (wave1<T>(eng)) return wave_toep_x<T, L, 1>(a, nb, s);
            return wave_toep_x<T, L, wave_lpl_default<T, L>()>(a, nb, s);
        }
    }
    if (a.pro == PRO_ARNOLDI) return hipErrorInvalidValue;   // wave engine only
    return stage_x_launch<T, L, KToepX>(a, nb, s, eng);
}

template <typename T, int L>
hipError_t toep_s_one(const ToepArgs<T>& a, int* nb, hipStream_t s, int eng) {
    if (a.g.n != L / 2 - 1) return hipErrorInvalidValue;   // the kernels take n = L/2 - 1
    if constexpr (column_engine_length<T, L>()) {
        if (eng == ENG_AUTO || eng == ENG_COL || eng == ENG_COLH) {
            static_assert(colx::TX == 2 * lines_per_block(L, false), "tile width");
            const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer);
            if (nb) *nb = g;
            if (!g) return hipSuccess;
            switch (a.epi) {
                case EPI_ADD_F:
                    hipLaunchKernelGGL((colx::k_col_toep<T, EPI_ADD_F>), dim3(g), dim3(colx::NT), 0, s, a);
                    break;
                case EPI_DOT_P:
                    hipLaunchKernelGGL((colx::k_col_toep<T, EPI_DOT_P>), dim3(g), dim3(colx::NT), 0, s, a);
                    break;
                case EPI_RESID:
                    hipLaunchKernelGGL((colx::k_col_toep<T, EPI_RESID>), dim3(g), dim3(colx::NT), 0, s, a);
                    break;
                default:
                    hipLaunchKernelGGL((colx::k_col_toep<T, EPI_NONE>), dim3(g), dim3(colx::NT), 0, s, a);
            }
            return hipGetLastError();
        }
    }
    if constexpr (wave_engine_length<L>()) {
        if (!stage_engine(eng)) {
            if (wave1<T>(eng)) return wave_toep_s<T, L, 1>(a, nb, s);
            return wave_toep_s<T, L, wave_lpl_default<T, L>()>(a, nb, s);
        }
    }
    return stage_s_launch<T, L, KToepS>(a, nb, s, eng);
}

template <typename T, int L>
hipError_t dst_x_one(const DstArgs<T>& a, int* nb, hipStream_t s, int eng) {
    if (a.g.n != L / 2 - 1) return hipErrorInvalidValue;   // the kernels take n = L/2 - 1
    if constexpr (wave_engine_length<L>()) {
        if (!stage_engine(eng)) {
            if (wave1<T>(eng)) return wave_dst_x<T, L, 1>(a, nb, s);
            return wave_dst_x<T, L, wave_lpl_default<T, L>()>(a, nb, s);
        }
    }
    return stage_x_launch<T, L, KDstX>(a, nb, s, eng);
}

template <typename T, int L, bool SCALE>
hipError_t dst_s_one(const DstArgs<T>& a, int* nb, hipStream_t s, int eng) {
    if (a.g.n != L / 2 - 1) return hipErrorInvalidValue;   // the kernels take n = L/2 - 1
    if constexpr (column_engine_length<T, L>()) {
        // default: the odd-extension DST for the plain pass, the half-length
        // DST for the Lambda-scale pass (measured fastest at 255^3)
        const bool half = eng == ENG_COLH || (eng == ENG_AUTO && SCALE);
        if (eng == ENG_AUTO || eng == ENG_COL || eng == ENG_COLH) {
            static_assert(colx::TX == 2 * lines_per_block(L, false), "tile width");
            const int g = s_blocks<T>(L, a.g.P1, a.g.n_outer);
            if (nb) *nb = g;
            if (!g) return hipSuccess;
            if (half) hipLaunchKernelGGL((colx::k_col_dsth<SCALE>), dim3(g), dim3(colx::NT), 0, s, a);
            else hipLaunchKernelGGL((colx::k_col_dst<SCALE>), dim3(g), dim3(colx::NT), 0, s, a);
            return hipGetLastError();
        }
    }
    if constexpr (wave_engine_length<L>()) {
        // float64 Lambda-scale pass: the stage engine's half-length DST-I
        // by default (the wave engine's odd extension holds two wavefronts
        // per SIMD: 163 against 143 us at 255^3)
        constexpr bool stage_default = SCALE && sizeof(T) == 8;
        if (!stage_engine(eng) && !(stage_default && eng == ENG_AUTO)) {
            if (wave1<T>(eng)) return wave_dst_s<T, L, SCALE, 1>(a, nb, s);
            return wave_dst_s<T, L, SCALE, wave_lpl_default<T, L>()>(a, nb, s);
        }
    }
    if constexpr (SCALE) {
        // lengths with an even half take the half-length DST-I
        if constexpr (L >= 8 && (L / 2) % 2 == 0) return stage_dstsh_launch<T, L>(a, nb, s, eng);
        else return stage_s_launch<T, L, KDstsS>(a, nb, s, eng);
    } else {
        return stage_s_launch<T, L, KDstS>(a, nb, s, eng);
    }
}

#define FSD_W_CASE_TX(LL) case LL: return toep_x_one<FT, LL>(a, nb, s, eng);
#define FSD_W_CASE_TS(LL) case LL: return toep_s_one<FT, LL>(a, nb, s, eng);
#define FSD_W_CASE_DX(LL) case LL: return dst_x_one<FT, LL>(a, nb, s, eng);
#define FSD_W_CASE_DS(LL) case LL: return dst_s_one<FT, LL, false>(a, nb, s, eng);
#define FSD_W_CASE_DSS(LL) case LL: return dst_s_one<FT, LL, true>(a, nb, s, eng);

#define FSD_DEFINE_LAUNCHERS2(T)                                                              \
    template <>                                                                              \
    hipError_t launch_toep_x<T>(int L, const ToepArgs<T>& a, int* nb, hipStream_t s, int eng) {       \
        using FT = T;                                                                        \
        switch (L) { FSD_FOR_EACH_L(FSD_W_CASE_TX) default: return hipErrorInvalidValue; }   \
    }                                                                                        \
    template <>                                                                              \
    hipError_t launch_toep_s<T>(int L, const ToepArgs<T>& a, int* nb, hipStream_t s, int eng) {       \
        using FT = T;                                                                        \
        switch (L) { FSD_FOR_EACH_L(FSD_W_CASE_TS) default: return hipErrorInvalidValue; }   \
    }                                                                                        \
    template <>                                                                              \
    hipError_t launch_dst_x<T>(int L, const DstArgs<T>& a, int* nb, hipStream_t s, int eng) {       \
        using FT = T;                                                                        \
        switch (L) { FSD_FOR_EACH_L(FSD_W_CASE_DX) default: return hipErrorInvalidValue; }   \
    }                                                                                        \
    template <>                                                                              \
    hipError_t launch_dst_s<T>(int L, const DstArgs<T>& a, int* nb, hipStream_t s, int eng) {         \
        using FT = T;                                                                        \
        switch (L) { FSD_FOR_EACH_L(FSD_W_CASE_DS) default: return hipErrorInvalidValue; }   \
    }                                                                                        \
    template <>                                                                              \
    hipError_t launch_dsts_s<T>(int L, const DstArgs<T>& a, int* nb, hipStream_t s, int eng) {        \
        using FT = T;                                                                        \
        switch (L) { FSD_FOR_EACH_L(FSD_W_CASE_DSS) default: return hipErrorInvalidValue; }  \
    }

}  // namespace fsd
