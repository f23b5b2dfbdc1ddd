// Internal declarations shared by the host plan/solver code and the HIP
// kernels.  Not part of the public ABI (include/fsd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fsd {

constexpr int kMaxRestartHdr = 64;   // = kMaxRestart (declared before Ctrl)

// Device-resident solver state.  Written only by the single-workgroup scalar
// kernels (thread 0, vector stores); read by every kernel of a Krylov loop,
// which returns at once when `done` is set so that iterations enqueued after
// convergence cost a launch each and nothing else.
// Output stores of the line passes are non-temporal (streamed to HBM).  The
// passes are bound by VALU and LDS issue, so writing through while they
// compute is mostly hidden; with ordinary stores their dirty lines stay in
// the caches and are written back during the memory-bound Krylov kernels
// that follow (a 12-vector multi-dot took 168 instead of 128 us after a
// 266 MB write).  Measured on the 255^3 CN steps: float64 GMRES 26.8 -> 27.7
// steps/s, mixed precision 59.8 -> 60.5.
template <typename T>
__device__ inline void st_nt(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}
__device__ inline void st_nt2(float* p, float x, float y) {
    typedef float nt_f2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(nt_f2{x, y}, reinterpret_cast<nt_f2*>(p));
}

struct Ctrl {
    double bb;        // ||b||^2 (or ||P^{-1} b||^2 for left GMRES)
    double rr;        // ||r||^2 of the current residual
    double rz;        // (r, z) of PCG
    double pq;        // (p, A p)
    double alpha, beta;
    double thresh;    // tol^2 * bb: stop when rr <= thresh
    double tol2;
    int iters;        // iterations taken in the current solve
    int maxit;
    int done;         // 1: converged or stopped
    int status;       // fsd_status of the solve
    int first;        // PCG: next p-update is p = z
    int gm_j;         // GMRES: current Arnoldi column
    int gm_m;         // GMRES: restart length
    int gm_k;         // GMRES: columns in the current cycle
    double gm_beta;   // GMRES: ||r0|| of the current cycle
    double gm_hnext;  // GMRES: norm of the new basis vector before scaling
    double gm_scale;  // GMRES: 1 / gm_hnext
    double abs2;      // absolute floor of thresh (0: purely relative test)
    double gm_w2;     // GMRES: ||w||^2 before Gram-Schmidt
    double gm_wp2;    // GMRES: ||w'||^2 after the first Gram-Schmidt pass
    double gm_eta2;   // GMRES: second pass when ||w'||^2 <= gm_eta2 ||w||^2
    int gm_reorth;    // GMRES: the current step takes the second pass
    int gm_nreorth;   // GMRES: second passes taken in this solve
    int gm_rflag[kMaxRestartHdr];   // GMRES: second pass taken at column j (this cycle)
    // GMRES small dense state: H is (m+1) x m column-major, then cs, sn, g, y, h
    double gm[1];
};

constexpr int kMaxRestart = kMaxRestartHdr;
constexpr size_t kCtrlBytes = sizeof(Ctrl) + sizeof(double) * ((kMaxRestart + 1) * kMaxRestart
                                                        + 6 * (kMaxRestart + 1) + 64);

// Epilogue of the last matvec pass.
enum Epi : int {
    EPI_NONE = 0,
    EPI_ADD_F = 1,    // o1 += dt * F (F dense float64 input)
    EPI_DOT_P = 2,    // partial sums of (p, o1)
    EPI_RESID = 3,    // o1 = b - o1, partial sums of ||o1||^2
};

// Prologue of the first matvec pass (x axis).
enum Pro : int {
    PRO_NONE = 0,
    PRO_PUPDATE = 1,  // u = z + beta p (p = z when ctrl->first); p <- u
    PRO_SCALE = 2,    // u = scale * u_in, scale = ctrl->gm_scale (GMRES v_{j+1} = w / h)
    PRO_ARNOLDI = 3,  // u = (u_in - V_{nv-1}) - sum_{i<nv} c_i V_i, c_i = ctrl->gm[hoff + i]
                      // (GMRES Gram-Schmidt update, unnormalised); u -> pro_p and
                      // the block partial of ||u||^2 -> partials[blockIdx.x]
};

// Geometry of one pass over the padded internal layout.
// The internal layout of a grid function is [n3][n2][P1] with P1 = n1
// rounded up to a multiple of 32; columns x >= n1 hold zeros.
struct PassGeo {
    int n;            // line length (points along the pass axis)
    int P1;           // padded row pitch
    long estride;     // element stride along the line
    long ostride;     // stride between outer indices (strided passes)
    int n_outer;      // number of outer indices (strided passes)
    int nrows;        // number of rows (x pass)
    // dense (ABI) layout of F for EPI_ADD_F: index = x + n1 * (i*fr_i + o*fr_o)
    int n1;
    long fr_i, fr_o;
    // preconditioner scale (strided DST-scale-DST pass)
    int nx;           // n1 (lines with x >= n1 are padding)
};

template <typename T>
struct ToepArgs {
    PassGeo g;
    const T* u_fft;       // input transformed by the Toeplitz factor
    const T* u_sten;      // input of the tridiagonal stencil (may be null)
    T* o1;                // Toeplitz(u_fft) [+ A(u_sten)] with epilogue
    T* o2;                // A(u_fft) (may be null)
    const T* spec;        // circulant spectrum, interleaved (re, im), L entries, 1/L folded
    const T* tw;          // twiddles exp(-2 pi i e / L), interleaved, L entries
    int epi;
    const double* F;      // EPI_ADD_F
    double dt;
    const T* dot_p;       // EPI_DOT_P
    const T* b;           // EPI_RESID
    double* partials;     // one double per workgroup
    int pro;
    T* pro_p;             // PRO_PUPDATE: p (read and written); PRO_SCALE / PRO_ARNOLDI: output
    const T* gs_V;        // PRO_ARNOLDI: basis vectors V_0 .. V_{nv-1}, gs_ld apart
    long gs_ld;
    int gs_nv;
    int gs_hoff;          // PRO_ARNOLDI: offset of the coefficients in ctrl->gm
    const Ctrl* ctrl;     // may be null (no early exit, no beta)
};

template <typename T>
struct DstArgs {
    PassGeo g;
    const T* u;
    T* o;
    const T* tw;
    T c;                  // sqrt(2/(n+1)) / 2 per transform
    // scale pass: Lambda = a_last[k] * P + lc_last[k] * Q per line
    const T* a_last;      // eigenvalues of A_n on the pass axis
    const T* lc_last;     // c_i * tau eigenvalues on the pass axis
    const T* a1; const T* lc1;   // x axis factors
    const T* a2; const T* lc2;   // y axis factors (3D scale pass only)
    int dim;
    int half;             // scale pass: Lambda^{-1/2} (the two-sided system) instead of Lambda^{-1}
    double* partials;     // Parseval partials of (r, P^{-1} r)
    int pnorm;            // float64 scale passes: the partials are ||P^{-1} r||^2 (Parseval
                          // of the scaled spectrum) instead; with o null the stage engine's
                          // half-length scale pass leaves the partials only
    const Ctrl* ctrl;
};

// Float32 DST-I as a bf16 MFMA product (fsd_gdst.hip), axes with n <= 256.
struct GdstArgs {
    PassGeo g;
    const float* u;
    float* o;
    const void* frag;     // bf16 fragments of S (see fsd_gdst.hip)
    const float* a_last; const float* lc_last;
    const float* a1; const float* lc1;
    const float* a2; const float* lc2;
    int dim;
    int half;             // scale pass: Lambda^{-1/2} instead of Lambda^{-1}
    double* partials;     // Parseval partials (scale pass)
    const Ctrl* ctrl;
};
bool gdst_supported(int n);
hipError_t launch_gdst_row(const GdstArgs& a, hipStream_t s);
hipError_t launch_gdst_col(const GdstArgs& a, bool scale, int* nblocks, hipStream_t s);
int gdst_col_blocks(const PassGeo& g);

// ---------------------------------------------------------------- launchers
// Each launcher dispatches on the transform length L = 2(n+1) of the pass
// and on the engine (the tile shape) that runs it:
//   ENG_AUTO        the default choice per length (below);
//   ENG_WAVE        wave engine (lengths 64..512; fsd_wave.hpp);
//   ENG_COL         column engine (float32 strided passes of length 512;
//                   fsd_cols.hpp), the DST by the odd extension;
//   ENG_COLH        column engine with the half-length DST-I (DST passes);
//   ENG_STAGE       LDS-stage engine, lines_per_block lines per tile;
//   ENG_STAGE_HALF  LDS-stage engine, half as many lines per tile;
//   ENG_WAVE1       wave engine with one complex line per lane group
//                   (float32; twice the wavefronts of ENG_WAVE).
// Defaults: column engine for float32 strided passes of length 512 (the
// half-length DST for the Lambda-scale pass), the stage engine for the
// float64 Lambda-scale pass (half-length DST), the wave engine for the
// other passes of lengths 64..512, the stage engine otherwise.  The stage
// engine's Lambda-scale pass takes the half-length DST-I wherever n + 1 is
// even.  An engine a length does not have falls back to the default.
enum Engine : int { ENG_AUTO = 0, ENG_WAVE = 1, ENG_COL = 2, ENG_COLH = 3, ENG_STAGE = 4,
                    ENG_STAGE_HALF = 5, ENG_WAVE1 = 6, ENG_COUNT = 7 };

template <typename T> hipError_t launch_toep_x(int L, const ToepArgs<T>& a, int* nblocks, hipStream_t s,
                                               int eng = ENG_AUTO);
template <typename T> hipError_t launch_toep_s(int L, const ToepArgs<T>& a, int* nblocks, hipStream_t s,
                                               int eng = ENG_AUTO);
template <typename T> hipError_t launch_dst_x(int L, const DstArgs<T>& a, int* nblocks, hipStream_t s,
                                              int eng = ENG_AUTO);
template <typename T> hipError_t launch_dst_s(int L, const DstArgs<T>& a, int* nblocks, hipStream_t s,
                                              int eng = ENG_AUTO);
template <typename T> hipError_t launch_dsts_s(int L, const DstArgs<T>& a, int* nblocks, hipStream_t s,
                                               int eng = ENG_AUTO);
// Engines that run a pass of length L (first: the default).
enum PassOp : int { OP_TOEP_X = 0, OP_TOEP_S = 1, OP_DST_X = 2, OP_DST_S = 3, OP_DSTS_S = 4 };
int pass_engines(int op, int L, bool f32, int* out);

// Complex lines per workgroup tile for transform length L (two real lines
// each).  Sized so one tile plus its twiddle table stays below 80 KB of LDS
// at L = 512, leaving room for two workgroups per CU (160 KB).  Lines
// longer than 2048 (n + 1 = 1536 .. 4096) take one or two lines per tile,
// with the twiddles read from the global table (L1-resident) instead of
// LDS: at L = 8192 one float64 line alone fills 139 KB of LDS.
__host__ __device__ constexpr int lines_per_block(int L, bool fp64) {
    return L > 2048 ? (fp64 || L > 4096 ? 1 : 2)
         : fp64 ? (L <= 512 ? 8 : (L <= 1024 ? 4 : 2)) : (L <= 512 ? 16 : (L <= 1024 ? 8 : 4));
}

// Twiddle table of the LDS-stage engine held in LDS (else read from the
// global table).
__host__ __device__ constexpr bool twiddles_in_lds(int L) { return L <= 2048; }

// Threads per workgroup tile: about one radix-8 butterfly per thread per
// stage (NCL * L / 8), rounded down to a power of two in [64, 512].
__host__ __device__ constexpr int threads_for_lines(int L, int ncl) {
    int w = ncl * L / 8;
    int t = 64;
    while (t * 2 <= w && t < 512) t *= 2;
    return t;
}
__host__ __device__ constexpr int threads_per_block(int L, bool fp64) {
    return threads_for_lines(L, lines_per_block(L, fp64));
}

// Transform lengths with a compiled plan: L = 2(n+1) in {2^a, 3*2^a}, 4..8192.
inline bool length_supported(int L) {
    switch (L) {
        case 4: case 6: case 8: case 12: case 16: case 24: case 32: case 48: case 64:
        case 96: case 128: case 192: case 256: case 384: case 512: case 768: case 1024:
        case 1536: case 2048: case 3072: case 4096: case 6144: case 8192:
            return true;
        default:
            return false;
    }
}

}  // namespace fsd
