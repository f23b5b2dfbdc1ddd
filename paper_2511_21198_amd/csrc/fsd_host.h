// Host-side problem state (plan, workspace layout, device pointers).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "../../include/fsd.h"
#include "fsd_internal.h"

namespace fsd {

struct Axis {
    int n = 0, L = 0;
    double h = 0, delta = 0, kp = 0, km = 0, eta = 0;
    std::vector<long double> q;        // q_0..q_n
    std::vector<double> aeig, lam;     // A_n and tau(H(T_n)) eigenvalues, k = 1..n
    std::vector<double> specA, specR;  // pass spectra for A and for the right-hand side
    std::vector<double> tw;            // twiddles exp(-2 pi i e/L), interleaved
    // circulant comparators (FSD_PC_TCHAN / FSD_PC_STRANG), interleaved complex
    int cM = 0, clog = 0;              // Bluestein FFT length (power of two >= 2n - 1), log2
    std::vector<double> ceA, ceB;      // eigenvalues of C(A_n) and of eta C(B_n), n each
    std::vector<double> cw;            // chirp exp(-i pi j^2 / n), j < n
    std::vector<double> cbsp;          // M-point spectrum of the conjugated chirp, bit-reversed
    std::vector<double> ctw;           // exp(-2 pi i k / M), k < M/2
};

// Records msg as the thread's last error (fsd_last_error) and returns s.
fsd_status set_error(fsd_status s, const std::string& msg);

void q_coefficients(double delta, int n, std::vector<long double>& q);
void axis_setup(Axis& ax, int n, double a, double b, double delta, double kp, double km, double dt);
void axis_spectra(Axis& ax, int axis_index);
void axis_circulant(Axis& ax, int kind);

template <typename T>
struct Tables {
    T* tw[3] = {nullptr, nullptr, nullptr};
    T* specA[3] = {nullptr, nullptr, nullptr};
    T* specR[3] = {nullptr, nullptr, nullptr};
    T* a[3] = {nullptr, nullptr, nullptr};    // A_n eigenvalues
    T* lc[3] = {nullptr, nullptr, nullptr};   // eta_i (k+ + k-) * tau eigenvalues
    void* sfrag[3] = {nullptr, nullptr, nullptr};  // bf16 MFMA fragments of S (float32, n <= 256)
};

template <typename T>
struct Vecs {
    T* x = nullptr;
    T* r = nullptr;
    T* p = nullptr;
    T* q = nullptr;
    T* z = nullptr;
    T* b = nullptr;
    T* t[4] = {nullptr, nullptr, nullptr, nullptr};
    T* up = nullptr;  // previous u_prev (time history for extrapolation)
    T* V = nullptr;   // GMRES basis, (restart + 1) vectors
    T* w = nullptr;   // GMRES work vector
};

}  // namespace fsd

namespace fsd {
// One profiled launch: hipEvents recorded on the problem's stream around a
// kernel, with the algorithmic bytes that launch moves.
// tag: Krylov iteration the launch belongs to (-1: none); skip: the launch
// returned at once because the solve had already stopped (not counted).
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes;
    int tag;
    bool skip;
};
}  // namespace fsd

struct fsd_problem_s {
    fsd_params p{};
    int dim = 3;
    fsd::Axis ax[3];
    int P1 = 0;           // padded pitch (n1 rounded up to 32)
    long rows = 0;        // n2 * n3
    long Np = 0;          // P1 * rows (padded vector length)
    long N = 0;           // n1 * n2 * n3
    bool symmetric = false;
    int solver = FSD_SOLVER_PCG;
    bool mixed = false;
    bool gdst[3] = {false, false, false};   // float32 DST-I on the matrix cores, per axis
    int restart = 20;
    int maxparts = 0;     // partial sums per reduction slot
    size_t ws_bytes = 0;

    bool bound = false;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    fsd::Ctrl* ctrl = nullptr;
    double* partials = nullptr;
    fsd::Tables<double> t64;
    fsd::Tables<float> t32;
    fsd::Vecs<double> v64;
    fsd::Vecs<float> v32;
    fsd::Ctrl* h_ctrl = nullptr;   // pinned host mirror of the ctrl header
    int last_iters = 4;
    int last_inner_iters[4] = {4, 4, 4, 4};   // per defect-correction pass (capped at 3)
    bool have_hist = false;
    // fsd_cn_step from u^{m-1}: the first residual of the solve, b - A x with
    // x = the packed u^{m-1} that b was built from (and F), is
    // 2 (b - A_N x) - dt F (resid_prev); taken once by first_residual
    bool r0_hint = false;
    const double* r0_F = nullptr;
    // comparator preconditioners (fsd_precond): complex work vector (Np
    // interleaved values) and per-axis tables of the circulant passes
    int pc = FSD_PC_TAU;
    double* zc = nullptr;
    double* cw[3] = {nullptr, nullptr, nullptr};
    double* cbsp[3] = {nullptr, nullptr, nullptr};
    double* ctw[3] = {nullptr, nullptr, nullptr};
    double* cea[3] = {nullptr, nullptr, nullptr};
    double* ceb[3] = {nullptr, nullptr, nullptr};

    // engine (tile shape) of each line pass, per precision (0: float64,
    // 1: float32) and pass kind (the profiler's kinds K_TOEP_X..K_DSTS_Z);
    // ENG_AUTO until fsd_autotune.  tune_kind >= 0 runs only that pass, with
    // engine tune_eng (the autotuner's timing runs).
    int eng[2][16] = {};
    int tune_kind = -1, tune_eng = 0;
    // executable graphs of Krylov iteration chunks (fsd_set_graphs): key,
    // graph; captured on first use, dropped when the workspace is rebound
    bool use_graphs = false;
    std::vector<std::pair<int, hipGraphExec_t>> graphs;

    bool prof_on = false;
    std::vector<fsd::ProfRec> prof;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_next = 0;
    int prof_tag = -1;
};
