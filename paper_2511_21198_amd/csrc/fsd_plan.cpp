// Host-side coefficients and transform plans (no device work).
//
//  * s_k, q_k:  Section 2 (``coef_expression``): q_0 = -s_0, q_k = s_{k-1} - s_k,
//    s_k a second difference of (k + 1/2 - j)^delta.  q_k is a third difference
//    of x^delta and loses about log10(k^3) digits when formed directly, so for
//    k >= 8 it is summed from the binomial expansion around kappa = k - 1:
//      q_k = kappa^delta * sum_{m odd >= 3} C(delta, m) (6 / 2^m - 2 (3/2)^m) kappa^{-m},
//    which follows from writing q_k = -(k+1/2)^d + 3(k-1/2)^d - 3(k-3/2)^d + (k-5/2)^d
//    and expanding each power in 1/kappa (the even moments cancel).  Small k
//    use the direct formula in long double.
//  * eta_i = dt / (2 Gamma(delta_i + 1) h_i^(2 - delta_i))  (Section 2).
//  * Eigenvalues of A_n: (3 + cos(k pi/(n+1)))/4 (Lemma 3.1, A_n is a tau matrix).
//  * Eigenvalues of tau(H(T_n)): q_1 + (q_0 + q_2) cos t_k + sum_{j=2}^{n-1} q_{j+1} cos(j t_k),
//    t_k = k pi/(n+1) (Lemma 3.2, summation index read as j).
//  * Circulant spectra: the Toeplitz factor applied on each axis pass is
//    embedded in a circulant of length L = 2(n+1) >= 2n-1 whose first column
//    is [col_0..col_{n-1}, 0, .., 0, row_{n-1}..row_1]; its DFT (scaled by 1/L)
//    is what the pass multiplies by.
#include <cmath>
#include <vector>

#include "fsd_host.h"

namespace fsd {

static long double s_direct(long double d, long k) {
    const long double h = 0.5L;
    if (k == 0) return powl(h, d);
    if (k == 1) return powl(3.0L * h, d) - 2.0L * powl(h, d);
    const long double kk = (long double)k;
    return powl(kk + h, d) - 2.0L * powl(kk - h, d) + powl(kk - 3.0L * h, d);
}

static long double q_series(long double d, long k) {
    const long double kap = (long double)(k - 1);
    const long double inv = 1.0L / kap;
    long double binom = 1.0L;    // C(d, m)
    long double ipow = 1.0L;     // kappa^{-m}
    long double p2 = 1.0L;       // 2^{-m}
    long double p32 = 1.0L;      // (3/2)^m
    long double sum = 0.0L;
    for (int m = 1; m <= 80; ++m) {
        binom *= (d - (long double)(m - 1)) / (long double)m;
        ipow *= inv;
        p2 *= 0.5L;
        p32 *= 1.5L;
        if (m % 2 == 1 && m >= 3) {
            const long double t = binom * (6.0L * p2 - 2.0L * p32) * ipow;
            sum += t;
            if (fabsl(t) <= 1e-24L * fabsl(sum)) break;
        }
    }
    return powl(kap, d) * sum;
}

void q_coefficients(double delta, int n, std::vector<long double>& q) {
    const long double d = (long double)delta;
    q.assign((size_t)n + 1, 0.0L);
    q[0] = -s_direct(d, 0);
    for (long k = 1; k <= n; ++k) {
        if (k < 8 || delta == 0.0)
            q[k] = s_direct(d, k - 1) - s_direct(d, k);
        else
            q[k] = q_series(d, k);
    }
}

void axis_setup(Axis& ax, int n, double a, double b, double delta, double kp, double km,
                double dt) {
    ax.n = n;
    ax.L = 2 * (n + 1);
    ax.delta = delta;
    ax.kp = kp;
    ax.km = km;
    ax.h = (b - a) / (double)(n + 1);
    ax.eta = (double)((long double)dt /
                      (2.0L * tgammal((long double)delta + 1.0L) *
                       powl((long double)ax.h, 2.0L - (long double)delta)));
    q_coefficients(delta, n, ax.q);

    // eigenvalues in the DST-I basis, k = 1..n
    const int L = ax.L;
    std::vector<long double> cosL((size_t)L);
    for (int e = 0; e < L; ++e) cosL[e] = cosl(2.0L * 3.14159265358979323846264338327950288L * e / L);
    ax.aeig.resize(n);
    ax.lam.resize(n);
    for (int k = 1; k <= n; ++k) {
        // cos(j k pi/(n+1)) = cos(2 pi (j k mod L) / L)
        ax.aeig[k - 1] = (double)((3.0L + cosL[k % L]) / 4.0L);
        long double lam = ax.q[1];
        if (n >= 2) lam += (ax.q[0] + ax.q[2]) * cosL[k % L];
        for (int j = 2; j <= n - 1; ++j) lam += ax.q[j + 1] * cosL[((long)j * k) % L];
        ax.lam[k - 1] = (double)lam;
    }
}

// First column / row of B = k+ T + k- T^T (Section 2, ``stiff_matrix``):
// column [(k+ + k-) q1, k+ q2 + k- q0, k+ q3, ..., k+ qn],
// row    [(k+ + k-) q1, k+ q0 + k- q2, k- q3, ..., k- qn].
static void b_col_row(const Axis& ax, std::vector<long double>& col, std::vector<long double>& row) {
    const int n = ax.n;
    const long double kp = ax.kp, km = ax.km;
    col.assign(n, 0.0L);
    row.assign(n, 0.0L);
    col[0] = row[0] = (kp + km) * ax.q[1];
    if (n >= 2) {
        col[1] = kp * ax.q[2] + km * ax.q[0];
        row[1] = kp * ax.q[0] + km * ax.q[2];
    }
    for (int j = 2; j < n; ++j) {
        col[j] = kp * ax.q[j + 1];
        row[j] = km * ax.q[j + 1];
    }
}

// Spectrum (1/L) DFT of the circulant embedding of the Toeplitz matrix
// c_a A_n + c_b B_n, interleaved (re, im).
static void toeplitz_spectrum(const Axis& ax, long double c_a, long double c_b, std::vector<double>& spec) {
    const int n = ax.n, L = ax.L;
    std::vector<long double> col, row;
    b_col_row(ax, col, row);
    for (int j = 0; j < n; ++j) { col[j] *= c_b; row[j] *= c_b; }
    col[0] += c_a * 0.75L;
    row[0] += c_a * 0.75L;
    if (n >= 2) { col[1] += c_a * 0.125L; row[1] += c_a * 0.125L; }
    std::vector<long double> e((size_t)L, 0.0L);
    for (int j = 0; j < n; ++j) e[j] = col[j];
    for (int j = 1; j < n; ++j) e[L - j] = row[j];
    const long double tp = 2.0L * 3.14159265358979323846264338327950288L;
    std::vector<long double> cs((size_t)L), sn((size_t)L);
    for (int m = 0; m < L; ++m) { cs[m] = cosl(tp * m / L); sn[m] = sinl(tp * m / L); }
    spec.assign(2 * (size_t)L, 0.0);
    for (int f = 0; f < L; ++f) {
        long double re = 0, im = 0;
        for (int j = 0; j < L; ++j) {
            if (e[j] == 0.0L) continue;
            const int m = (int)(((long)j * f) % L);
            re += e[j] * cs[m];
            im -= e[j] * sn[m];
        }
        spec[2 * f] = (double)(re / L);
        spec[2 * f + 1] = (double)(im / L);
    }
}

void axis_spectra(Axis& ax, int axis_index) {
    // x pass applies (A1 + s eta1 B1); y and z passes apply s eta_i B_i (the
    // A_i stencil is added separately); s = +1 for A, -1 for the right-hand side.
    const long double ca = axis_index == 0 ? 1.0L : 0.0L;
    toeplitz_spectrum(ax, ca, (long double)ax.eta, ax.specA);
    toeplitz_spectrum(ax, ca, -(long double)ax.eta, ax.specR);
    const int L = ax.L;
    const long double tp = 2.0L * 3.14159265358979323846264338327950288L;
    ax.tw.resize(2 * (size_t)L);
    for (int e = 0; e < L; ++e) {
        ax.tw[2 * e] = (double)cosl(tp * e / L);
        ax.tw[2 * e + 1] = (double)(-sinl(tp * e / L));
    }
}

// ------------------------------------------------------------ circulant comparators
// Section 4 compares the method with T. Chan's and Strang's circulant
// preconditioners: every Toeplitz factor (A_n and B_n) is replaced by its
// circulant approximation.  For a Toeplitz matrix with entries t_{j-k}
// (textbook definitions, cited but not restated by the paper):
//   T. Chan:  c_j = ((n - j) t_j + j t_{j-n}) / n   (nearest in Frobenius norm)
//   Strang:   s_j = t_j for j <= n/2, t_{j-n} for j > n/2 (central diagonals)
// A circulant with first column c has eigenvalues sum_j c_j e^{-2 pi i j k/n}
// in the DFT basis.  The DFT of length n (odd for n = 2^a - 1) is taken by
// Bluestein's chirp transform: X_k = w_k sum_j (x_j w_j) conj(w_{k-j}) with
// w_j = e^{-i pi j^2 / n}, a convolution done by FFTs of a power-of-two
// length M >= 2n - 1.
static void circ_column(const std::vector<long double>& col, const std::vector<long double>& row,
                        int kind, std::vector<long double>& c) {
    const int n = (int)col.size();
    c.assign(n, 0.0L);
    for (int j = 0; j < n; ++j) {
        const long double tp = col[j];                     // t_j
        const long double tn = j > 0 ? row[n - j] : 0.0L;  // t_{j-n}
        if (kind == FSD_PC_STRANG)
            c[j] = j <= n / 2 ? tp : tn;
        else
            c[j] = ((long double)(n - j) * tp + (long double)j * tn) / (long double)n;
    }
}

static void circ_eigs(const std::vector<long double>& c, long double scale, std::vector<double>& out) {
    const int n = (int)c.size();
    const long double tp = 2.0L * 3.14159265358979323846264338327950288L;
    std::vector<long double> cs(n), sn(n);
    for (int m = 0; m < n; ++m) {
        cs[m] = cosl(tp * m / n);
        sn[m] = sinl(tp * m / n);
    }
    out.assign(2 * (size_t)n, 0.0);
    for (int k = 0; k < n; ++k) {
        long double re = 0.0L, im = 0.0L;
        for (int j = 0; j < n; ++j) {
            const int e = (int)(((long)j * k) % n);
            re += c[j] * cs[e];
            im -= c[j] * sn[e];
        }
        out[2 * k] = (double)(scale * re);
        out[2 * k + 1] = (double)(scale * im);
    }
}

static int bit_reverse(int k, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((k >> b) & 1) << (bits - 1 - b);
    return r;
}

void axis_circulant(Axis& ax, int kind) {
    const int n = ax.n;
    std::vector<long double> acol(n, 0.0L), arow(n, 0.0L);   // A_n = tridiag(1, 6, 1) / 8
    acol[0] = arow[0] = 0.75L;
    if (n >= 2) acol[1] = arow[1] = 0.125L;
    std::vector<long double> bcol, brow, c;
    b_col_row(ax, bcol, brow);
    circ_column(acol, arow, kind, c);
    circ_eigs(c, 1.0L, ax.ceA);
    circ_column(bcol, brow, kind, c);
    circ_eigs(c, (long double)ax.eta, ax.ceB);

    int M = 2, lg = 1;
    while (M < 2 * n - 1) { M <<= 1; ++lg; }
    ax.cM = M;
    ax.clog = lg;
    const long double pi = 3.14159265358979323846264338327950288L;
    std::vector<long double> wr(n), wi(n);
    ax.cw.assign(2 * (size_t)n, 0.0);
    for (int j = 0; j < n; ++j) {
        const long m = ((long)j * j) % (2L * n);   // e^{-i pi j^2/n} has period 2n in j^2
        wr[j] = cosl(pi * m / n);
        wi[j] = -sinl(pi * m / n);
        ax.cw[2 * j] = (double)wr[j];
        ax.cw[2 * j + 1] = (double)wi[j];
    }
    // b_m = conj(w_m) for |m| < n, wrapped to length M
    std::vector<long double> br(M, 0.0L), bi(M, 0.0L);
    for (int m = 0; m < n; ++m) {
        br[m] = wr[m];
        bi[m] = -wi[m];
        if (m > 0) { br[M - m] = wr[m]; bi[M - m] = -wi[m]; }
    }
    std::vector<long double> cm(M), sm(M);
    for (int e = 0; e < M; ++e) {
        cm[e] = cosl(2.0L * pi * e / M);
        sm[e] = sinl(2.0L * pi * e / M);
    }
    ax.cbsp.assign(2 * (size_t)M, 0.0);
    for (int k = 0; k < M; ++k) {
        long double re = 0.0L, im = 0.0L;
        for (int m = 0; m < M; ++m) {
            if (br[m] == 0.0L && bi[m] == 0.0L) continue;
            const int e = (int)(((long)m * k) % M);
            re += br[m] * cm[e] + bi[m] * sm[e];
            im += bi[m] * cm[e] - br[m] * sm[e];
        }
        const int p = bit_reverse(k, lg);
        ax.cbsp[2 * p] = (double)re;
        ax.cbsp[2 * p + 1] = (double)im;
    }
    ax.ctw.assign((size_t)M, 0.0);   // M/2 complex
    for (int k = 0; k < M / 2; ++k) {
        ax.ctw[2 * k] = (double)cm[k];
        ax.ctw[2 * k + 1] = (double)(-sm[k]);
    }
}

}  // namespace fsd
