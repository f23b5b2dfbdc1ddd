// Host launchers of the GMRES kernels (fsd_gmres.hip).
#pragma once

#include "fsd_internal.h"

namespace fsd {

constexpr int kGmGrid = 1024;

// k_maxpy modes
enum MaxpyMode : int { MX_NORM = 0, MX_DOTS = 1, MX_REORTH = 2 };

enum GmOp : int {
    GM_PBB = 0,    // bb = ||P^{-1} b||^2, thresh = tol^2 bb
    GM_BETA = 1,   // beta = ||r0||, g = beta e1, scale = 1/beta (done if small)
    GM_H1 = 2,     // H[0..j, j] = first Gram-Schmidt coefficients; ||w||^2
    GM_H2 = 3,     // reorthogonalisation test; if taken, second pass coefficients
                   // added to H[0..j, j] and kept in h2
    GM_STEP = 4,   // H[j+1, j] = ||w||, Givens rotations, residual test
    GM_SOLVE = 5,  // y = R^{-1} g for the k columns of the cycle
    GM_H2S = 6,    // GM_H2 then GM_STEP in one launch, for a zero reorthogonalisation
                   // threshold (no second pass between them)
    // Unnormalised basis (one Gram-Schmidt pass, the update of v_{j+1} fused
    // into the next matvec's x pass): V_i holds v_i / s_i, s_i = 1/||V_i||
    // kept in ctrl->gm (s_0 = 1).
    GM_COEF = 7,   // H[0..j, j] and the coefficients c_i = s_i^2 V_i^T (w - V_j) from
                   // the multi-dot partials
    GM_NEXT = 8,   // ||V_j||^2 from the partials (row nv): s_j, H[j, j-1], Givens
                   // rotations and residual test of column j - 1
};

// Offsets inside Ctrl::gm for restart m.
inline int gm_off_h2(int m) { return (m + 1) * m + m + m + (m + 1) + m; }
inline int gm_off_y(int m) { return (m + 1) * m + m + m + (m + 1); }

int gm_grid(long N);

template <typename T>
hipError_t gm_mdot(const T* V, long ld, int nv, const T* w, long N, double* partials,
                   const Ctrl* ctrl, int* nparts, hipStream_t s);
template <typename T>
hipError_t gm_maxpy(const T* V, long ld, int nv, const T* in, T* out, long N, const Ctrl* ctrl,
                    int hoff, int mode, double* partials, int* nparts, hipStream_t s);
// x += V y, or x = V y with overwrite (x not read)
template <typename T>
hipError_t gm_update(T* x, const T* V, long ld, long N, int kmax, const Ctrl* ctrl, int yoff,
                     hipStream_t s, bool overwrite = false);
template <typename T>
hipError_t gm_scale(const T* in, T* out, long N, const Ctrl* ctrl, hipStream_t s);
// GM_PBB / GM_BETA with nparts = 0 take the squared norm val instead of a
// sum of partials.
hipError_t gm_scalar(Ctrl* c, const double* partials, int nparts, int nv, int j, int op,
                     hipStream_t s, double val = 0.0);
hipError_t gm_restart(Ctrl* c, hipStream_t s);

}  // namespace fsd
