/*
 * sphfilt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU definition of the double FFT filter
 * (arXiv:2305.01537, Sec. II.A "Filtering algorithms").  It exists so that the
 * GPU library can be checked against something written straight from the
 * paper.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product library never links or calls it, and it
 * shares no source with the GPU path.
 *
 * What it computes, in the paper's order and notation:
 *   Theta-pass (Sec. II.A, extension equation and the theta FFT filter):
 *     for every field f, shell i and meridian k < n_phi/2 build the
 *     2pi-periodic line  g(vartheta) = X(theta, phi_k)            on [0, pi]
 *                                     = (-1)^a X(2pi - vartheta, phi_k + pi) on [pi, 2pi],
 *     take its DFT, multiply mode l by f(|l|, l_max), take the inverse DFT and
 *     write the two halves back to meridians k and k + n_phi/2.
 *   Phi-pass (the phi FFT filter that follows): for every ring (f, i, j) take
 *     the DFT along phi, multiply mode m by f(|m|, m_max(theta_j)), invert.
 *   Forward filter = phi-pass after theta-pass (the paper filters in theta
 *   first, then in phi).  Adjoint = theta-pass after phi-pass, because each
 *   pass is a real symmetric operator.
 *   Cutoffs (Sec. II.A, the l_max / m_max equations):
 *     l_max = max(floor, 2 rho L),  m_max = max(floor, 2 rho sin(theta_j) L),
 *     with rho = r / dr_min and floor = 2 in the paper.
 *   Masks: exponential filter (eq. exp_filter), Gaussian filter
 *     (eq. gaussian_filter) and the spectrally sharp low-pass the paper
 *     mentions beside them.
 *   Hybrid filter (the automatic switch at the end of Sec. II.A): for each
 *     extended theta line and each phi ring of a field, Jameson's shock
 *     detector sigma_i = |u_{i-1} - 2 u_i + u_{i+1}| /
 *     (|u_{i-1}| + 2|u_i| + |u_{i+1}| + eps) is evaluated at every cell
 *     (periodic neighbours along the line); if any cell has
 *     sigma >= threshold (0.95 in the paper) the line takes the Gaussian
 *     filter, otherwise the exponential one.
 *
 * Every DFT here is the direct O(N^2) sum with the angle index reduced
 * exactly, (q*n) mod N, before the table lookup.  Nothing is skipped: lines
 * whose mask is all ones are still transformed.
 *
 * Readings of the paper that this file fixes (see the design notes):
 *   grid: theta_j = (j + 1/2) pi / n_theta, phi_k = 2 pi k / n_phi;
 *   the extended half maps row n >= n_theta to row 2 n_theta - 1 - n;
 *   masks depend on |l| (both signs), cutoffs are real (not rounded);
 *   sin(theta_j) is evaluated at the mirror-symmetric angle
 *   (min(j, n_theta-1-j) + 1/2) pi / n_theta, which is the same number;
 *   forward DFT unnormalised, inverse scaled by 1/N.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXP   0
#define ORC_GAUSS 1
#define ORC_SHARP 2
#define ORC_HYBRID 3

#define ORC_OK     0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* Detector parameters of the hybrid filter: epsilon and the threshold. */
static double orc_det_eps = 1e-12;
static double orc_det_threshold = 0.95;

void orc_set_detector(double eps, double threshold)
{
    orc_det_eps = eps;
    orc_det_threshold = threshold;
}

/* Threads of the parallel loops over lines (n <= 0: all processors); returns
 * the previous setting.  Only for timing the oracle: results do not depend on
 * it (each line is computed by one thread in a fixed order). */
int orc_set_threads(int n)
{
    const int prev = omp_get_max_threads();
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
    return prev;
}

/* Jameson's detector on one periodic line: 1 if any cell has sigma >= threshold. */
int orc_shock_detected(const double *g, int N)
{
    for (int n = 0; n < N; ++n) {
        const double a = g[(n - 1 + N) % N], b = g[n], c = g[(n + 1) % N];
        const double sigma = fabs(a - 2.0 * b + c) / (fabs(a) + 2.0 * fabs(b) + fabs(c) + orc_det_eps);
        if (sigma >= orc_det_threshold) return 1;
    }
    return 0;
}

/* Filter function f(qhat, c) for a mode of magnitude qhat and cutoff c. */
double orc_mask(int kind, double qhat, double c)
{
    switch (kind) {
    case ORC_EXP:   /* eq. exp_filter: 1 up to the cutoff, e^{-(|l|-l_max)} above */
        return qhat <= c ? 1.0 : exp(-(qhat - c));
    case ORC_GAUSS: /* eq. gaussian_filter: exp(log(0.9) (l/(l_max+1))^2) */
    {
        double u = qhat / (c + 1.0);
        return exp(log(0.9) * u * u);
    }
    case ORC_SHARP: /* sharp low-pass: keep modes up to the cutoff, drop the rest */
        return qhat <= c ? 1.0 : 0.0;
    default:
        return NAN;
    }
}

/* l_max of one shell: max(floor, 2 r/dr_min L). */
double orc_theta_cutoff(double rho, double L, double floor_modes)
{
    double c = 2.0 * rho * L;
    return c > floor_modes ? c : floor_modes;
}

/* sin(theta_j) at the cell-centred colatitude, evaluated on the northern mirror. */
double orc_sin_theta(int j, int n_theta)
{
    int jm = (j < n_theta - 1 - j) ? j : n_theta - 1 - j;
    return sin(((double)jm + 0.5) * ORC_PI / (double)n_theta);
}

/* m_max of one ring: max(floor, 2 r/dr_min sin(theta_j) L). */
double orc_phi_cutoff(double rho, double L, int j, int n_theta, double floor_modes)
{
    double c = 2.0 * rho * orc_sin_theta(j, n_theta) * L;
    return c > floor_modes ? c : floor_modes;
}

/*
 * Filter one real line g[0..N) into out[0..N):
 *   G[q]  = sum_n g[n] exp(-2 pi i (q n mod N) / N)
 *   G[q] *= f(qhat, c),  qhat = q for q <= N/2, else N - q
 *   out[n] = Re (1/N) sum_q G[q] exp(+2 pi i (q n mod N) / N)
 * The largest |Im| of the inverse is folded into *imag_max.
 * ct/st hold cos/sin(2 pi m / N) for m in [0, N).
 */
static void orc_filter_line(int N, const double *g, double *out, int kind, double c,
                            const double *ct, const double *st, double *Gre, double *Gim,
                            double *imag_max)
{
    for (int q = 0; q < N; ++q) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n < N; ++n) {
            int m = (int)(((int64_t)q * n) % N);
            re += g[n] * ct[m];
            im -= g[n] * st[m];
        }
        int qhat = (q <= N / 2) ? q : N - q;
        double f = orc_mask(kind, (double)qhat, c);
        Gre[q] = re * f;
        Gim[q] = im * f;
    }
    for (int n = 0; n < N; ++n) {
        double re = 0.0, im = 0.0;
        for (int q = 0; q < N; ++q) {
            int m = (int)(((int64_t)q * n) % N);
            re += Gre[q] * ct[m] - Gim[q] * st[m];
            im += Gre[q] * st[m] + Gim[q] * ct[m];
        }
        out[n] = re / (double)N;
        double a = fabs(im / (double)N);
        if (a > *imag_max) *imag_max = a;
    }
}

/* The extended line of meridian pair (k, k + n_phi/2) of one shell X:
 * g[n] = X[n][k] for n < n_theta, s X[2 n_theta - 1 - n][k + n_phi/2] after. */
static void orc_extended_line(const double *X, int k, int n_theta, int n_phi, double s, double *g)
{
    const int N = 2 * n_theta, half = n_phi / 2;
    for (int n = 0; n < n_theta; ++n) g[n] = X[(int64_t)n * n_phi + k];
    for (int n = n_theta; n < N; ++n) g[n] = s * X[(int64_t)(N - 1 - n) * n_phi + k + half];
}

static void orc_tables(int N, double *ct, double *st)
{
    for (int m = 0; m < N; ++m) {
        ct[m] = cos(2.0 * ORC_PI * (double)m / (double)N);
        st[m] = sin(2.0 * ORC_PI * (double)m / (double)N);
    }
}

static int orc_check(int n_fields, int n_r, int n_theta, int n_phi, const int *parity,
                     const double *rho, const double *L, const int *kind)
{
    if (n_fields <= 0 || n_r <= 0 || n_theta <= 0 || n_phi <= 0 || (n_phi & 1)) return ORC_EINVAL;
    if (!parity || !rho || !L || !kind) return ORC_EINVAL;
    for (int f = 0; f < n_fields; ++f) {
        if (parity[f] != 1 && parity[f] != -1) return ORC_EINVAL;
        if (kind[f] < ORC_EXP || kind[f] > ORC_HYBRID) return ORC_EINVAL;
    }
    return ORC_OK;
}

/*
 * Theta-pass over the whole array in[f][i][j][k] (C order, k fastest) into out.
 * One extended line per meridian pair (k, k + n_phi/2): one transform filters
 * both meridians (the paper's "double covering").
 */
int orc_theta_pass(const double *in, double *out, int n_fields, int n_r, int n_theta, int n_phi,
                   const int *parity, const double *rho, const double *L, const int *kind,
                   double floor_modes, double *imag_max_out)
{
    int rc = orc_check(n_fields, n_r, n_theta, n_phi, parity, rho, L, kind);
    if (rc) return rc;
    const int N = 2 * n_theta, half = n_phi / 2;
    double *ct = malloc(sizeof(double) * N), *st = malloc(sizeof(double) * N);
    if (!ct || !st) { free(ct); free(st); return ORC_ENOMEM; }
    orc_tables(N, ct, st);
    const int64_t n_lines = (int64_t)n_fields * n_r * half;
    double imag_max = 0.0;
    int fail = 0;
#pragma omp parallel reduction(max : imag_max) reduction(| : fail)
    {
        double *g = malloc(sizeof(double) * N), *o = malloc(sizeof(double) * N);
        double *Gre = malloc(sizeof(double) * N), *Gim = malloc(sizeof(double) * N);
        if (!g || !o || !Gre || !Gim) fail = 1;
#pragma omp for schedule(static)
        for (int64_t line = 0; line < n_lines; ++line) {
            if (fail) continue;
            int k = (int)(line % half);
            int i = (int)((line / half) % n_r);
            int f = (int)(line / ((int64_t)half * n_r));
            const double s = (double)parity[f];
            const double *X = in + ((int64_t)f * n_r + i) * (int64_t)n_theta * n_phi;
            double *Y = out + ((int64_t)f * n_r + i) * (int64_t)n_theta * n_phi;
            orc_extended_line(X, k, n_theta, n_phi, s, g);
            double c = orc_theta_cutoff(rho[i], L[f], floor_modes);
            int k_line = kind[f];
            if (k_line == ORC_HYBRID) k_line = orc_shock_detected(g, N) ? ORC_GAUSS : ORC_EXP;
            orc_filter_line(N, g, o, k_line, c, ct, st, Gre, Gim, &imag_max);
            for (int n = 0; n < n_theta; ++n) Y[(int64_t)n * n_phi + k] = o[n];
            for (int n = n_theta; n < N; ++n) Y[(int64_t)(N - 1 - n) * n_phi + k + half] = s * o[n];
        }
        free(g); free(o); free(Gre); free(Gim);
    }
    free(ct); free(st);
    if (imag_max_out) *imag_max_out = imag_max;
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* Phi-pass: every ring (f, i, j) filtered along phi with its own m_max. */
int orc_phi_pass(const double *in, double *out, int n_fields, int n_r, int n_theta, int n_phi,
                 const int *parity, const double *rho, const double *L, const int *kind,
                 double floor_modes, double *imag_max_out)
{
    int rc = orc_check(n_fields, n_r, n_theta, n_phi, parity, rho, L, kind);
    if (rc) return rc;
    const int N = n_phi;
    double *ct = malloc(sizeof(double) * N), *st = malloc(sizeof(double) * N);
    if (!ct || !st) { free(ct); free(st); return ORC_ENOMEM; }
    orc_tables(N, ct, st);
    const int64_t n_rings = (int64_t)n_fields * n_r * n_theta;
    double imag_max = 0.0;
    int fail = 0;
#pragma omp parallel reduction(max : imag_max) reduction(| : fail)
    {
        double *Gre = malloc(sizeof(double) * N), *Gim = malloc(sizeof(double) * N);
        if (!Gre || !Gim) fail = 1;
#pragma omp for schedule(static)
        for (int64_t ring = 0; ring < n_rings; ++ring) {
            if (fail) continue;
            int j = (int)(ring % n_theta);
            int i = (int)((ring / n_theta) % n_r);
            int f = (int)(ring / ((int64_t)n_theta * n_r));
            double c = orc_phi_cutoff(rho[i], L[f], j, n_theta, floor_modes);
            int k_line = kind[f];
            if (k_line == ORC_HYBRID)
                k_line = orc_shock_detected(in + ring * n_phi, N) ? ORC_GAUSS : ORC_EXP;
            orc_filter_line(N, in + ring * n_phi, out + ring * n_phi, k_line, c, ct, st, Gre,
                            Gim, &imag_max);
        }
        free(Gre); free(Gim);
    }
    free(ct); free(st);
    if (imag_max_out) *imag_max_out = imag_max;
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* Forward filter: theta-pass first, then phi-pass. */
int orc_forward(const double *in, double *out, int n_fields, int n_r, int n_theta, int n_phi,
                const int *parity, const double *rho, const double *L, const int *kind,
                double floor_modes, double *imag_max_out)
{
    size_t n = (size_t)n_fields * n_r * n_theta * n_phi;
    double *tmp = malloc(sizeof(double) * (n ? n : 1));
    if (!tmp) return ORC_ENOMEM;
    double a = 0.0, b = 0.0;
    int rc = orc_theta_pass(in, tmp, n_fields, n_r, n_theta, n_phi, parity, rho, L, kind,
                            floor_modes, &a);
    if (!rc)
        rc = orc_phi_pass(tmp, out, n_fields, n_r, n_theta, n_phi, parity, rho, L, kind,
                          floor_modes, &b);
    free(tmp);
    if (imag_max_out) *imag_max_out = a > b ? a : b;
    return rc;
}

/* Adjoint (transpose) of the forward filter: phi-pass first, then theta-pass. */
int orc_adjoint(const double *in, double *out, int n_fields, int n_r, int n_theta, int n_phi,
                const int *parity, const double *rho, const double *L, const int *kind,
                double floor_modes, double *imag_max_out)
{
    size_t n = (size_t)n_fields * n_r * n_theta * n_phi;
    double *tmp = malloc(sizeof(double) * (n ? n : 1));
    if (!tmp) return ORC_ENOMEM;
    double a = 0.0, b = 0.0;
    int rc = orc_phi_pass(in, tmp, n_fields, n_r, n_theta, n_phi, parity, rho, L, kind,
                          floor_modes, &a);
    if (!rc)
        rc = orc_theta_pass(tmp, out, n_fields, n_r, n_theta, n_phi, parity, rho, L, kind,
                            floor_modes, &b);
    free(tmp);
    if (imag_max_out) *imag_max_out = a > b ? a : b;
    return rc;
}

/* The hybrid filter's choices for one pass over `in`, without filtering:
 * theta: dec[(f n_r + i) n_phi/2 + k] for the extended line of meridian pair k;
 * phi:   dec[(f n_r + i) n_theta + j] for ring j.  1 = Gaussian, 0 = exponential.
 * Fields whose kind is not hybrid get 0. */
int orc_theta_decisions(const double *in, unsigned char *dec, int n_fields, int n_r, int n_theta,
                        int n_phi, const int *parity, const int *kind)
{
    if (n_fields <= 0 || n_r <= 0 || n_theta <= 0 || n_phi <= 0 || (n_phi & 1)) return ORC_EINVAL;
    const int N = 2 * n_theta, half = n_phi / 2;
    double *g = malloc(sizeof(double) * N);
    if (!g) return ORC_ENOMEM;
    for (int f = 0; f < n_fields; ++f)
        for (int i = 0; i < n_r; ++i)
            for (int k = 0; k < half; ++k) {
                const double s = (double)parity[f];
                const double *X = in + ((int64_t)f * n_r + i) * (int64_t)n_theta * n_phi;
                orc_extended_line(X, k, n_theta, n_phi, s, g);
                dec[((int64_t)f * n_r + i) * half + k] =
                    (unsigned char)(kind[f] == ORC_HYBRID && orc_shock_detected(g, N));
            }
    free(g);
    return ORC_OK;
}

int orc_phi_decisions(const double *in, unsigned char *dec, int n_fields, int n_r, int n_theta,
                      int n_phi, const int *kind)
{
    if (n_fields <= 0 || n_r <= 0 || n_theta <= 0 || n_phi <= 0) return ORC_EINVAL;
    const int64_t n_rings = (int64_t)n_fields * n_r * n_theta;
    for (int64_t ring = 0; ring < n_rings; ++ring) {
        const int f = (int)(ring / ((int64_t)n_theta * n_r));
        dec[ring] = (unsigned char)(kind[f] == ORC_HYBRID && orc_shock_detected(in + ring * n_phi, n_phi));
    }
    return ORC_OK;
}
