// Line passes of the circulant comparator preconditioners (Section 4):
// P^{-1} r = F^{-1} Lambda^{-1} F r with F the d-dimensional DFT of lengths
// n_i, taken axis by axis with Bluestein's chirp transform (float64).
#pragma once

#include <hip/hip_runtime.h>

#include "fsd_internal.h"

namespace fsd {

enum CircMode : int {
    CM_FWD_R2C = 0,   // real input, forward DFT, complex output (first axis)
    CM_FWD = 1,       // complex forward DFT (middle axis)
    CM_LAST = 2,      // forward DFT, divide by Lambda, inverse DFT (last axis)
    CM_INV = 3,       // complex inverse DFT with 1/n (middle axis)
    CM_INV_C2R = 4    // inverse DFT with 1/n, real part out (first axis)
};

struct CircArgs {
    const double* in_r = nullptr;    // CM_FWD_R2C input (padded real layout)
    const double2* in_c = nullptr;   // complex input (may equal out_c)
    double* out_r = nullptr;         // CM_INV_C2R output (padded real layout)
    double2* out_c = nullptr;
    long nlines = 0;                 // lines of the pass
    int nx = 1;                      // line l is (l / nx, l % nx) ...
    long os = 0, xs = 0;             // ... starting at (l / nx) * os + (l % nx) * xs
    long st = 1;                     // element stride along a line
    int n = 0;                       // line length
    int M = 2, logM = 1;             // Bluestein FFT length (power of two >= 2n - 1)
    int lpb = 1;                     // lines per workgroup
    int mode = CM_FWD;
    int pad = 0;                     // CM_INV_C2R: row pitch; columns [n, pad) are zeroed
    const double2* w = nullptr;      // chirp e^{-i pi j^2 / n}, j < n
    const double2* bsp = nullptr;    // M-point spectrum of the conjugated chirp, bit-reversed
    const double2* tw = nullptr;     // e^{-2 pi i k / M}, k < M/2
    // CM_LAST: Lambda = prod_i a_i + sum_i b_i prod_{j != i} a_j (b_i carries eta_i)
    const double2* ea[3] = {nullptr, nullptr, nullptr};
    const double2* eb[3] = {nullptr, nullptr, nullptr};
    int dim = 3;
    const Ctrl* ctrl = nullptr;      // skip the pass once ctrl->done (may be null)
};

// Workgroup shape of a pass with FFT length M: lines per workgroup (the
// LDS holds lpb * M <= 2048 complex line values and the M/2 twiddles).
int circ_lines_per_block(int M);

hipError_t launch_circ(const CircArgs& a, hipStream_t s);

}  // namespace fsd
