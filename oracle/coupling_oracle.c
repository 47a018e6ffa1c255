/*
 * coupling_oracle.c -- plain FP64 CPU oracle for the NNP-MM coupling term.
 *
 * TEST INFRASTRUCTURE ONLY (see nnp_oracle.c): nothing on the product path
 * may include, link or call it.  It shares no code with the HIP library.
 *
 * Mechanical embedding (Methods, Eq. 4): the coupling energy is the double
 * sum over NNP atoms i and MM atoms j of a Coulomb term and a 12-6
 * Lennard-Jones term,
 *
 *   V = sum_i sum_j [ k q_i q_j / r_ij
 *                     + 4 eps_ij ((sigma_ij / r_ij)^12 - (sigma_ij / r_ij)^6) ]
 *
 * with k = 1 / (4 pi eps0) in the caller's units.  Readings: the pair
 * parameters follow the Lorentz-Berthelot rules, sigma_ij = (sigma_i +
 * sigma_j) / 2 and eps_ij = sqrt(eps_i eps_j); an optional plain cutoff
 * (cutoff > 0) drops every pair with r_ij >= cutoff (no switching).
 * Forces are F = -dV/dx on both sides, by the exact derivative of each pair
 * term along the pair's unit vector.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* energy and dV/dr of one pair */
static void pair_term(double k, double qi, double qj, double si, double sj, double ei,
                      double ej, double r, double* v, double* dv_dr)
{
    const double sig = 0.5 * (si + sj);
    const double eps = sqrt(ei * ej);
    const double coul = k * qi * qj / r;
    const double sr6 = pow(sig / r, 6.0);
    const double sr12 = sr6 * sr6;
    *v = coul + 4.0 * eps * (sr12 - sr6);
    *dv_dr = -coul / r + 4.0 * eps * (-12.0 * sr12 + 6.0 * sr6) / r;
}

/* x_*: [n][3]; par_*: [n][3] = (q, sigma, eps).  E is the coupling energy;
 * F_nnp, F_mm ([n][3]) are overwritten.  abs_sum (if non-NULL) receives
 * sum over pairs of |v_ij| (a scale for rounding-error bounds). */
void orc_coupling(int32_t n_nnp, const double* x_nnp, const double* par_nnp, int32_t n_mm,
                  const double* x_mm, const double* par_mm, double k, double cutoff,
                  double* E, double* F_nnp, double* F_mm, double* abs_sum)
{
    double e = 0.0, a = 0.0;
    memset(F_nnp, 0, sizeof(double) * 3 * (size_t)n_nnp);
    memset(F_mm, 0, sizeof(double) * 3 * (size_t)n_mm);
    for (int i = 0; i < n_nnp; ++i)
        for (int j = 0; j < n_mm; ++j) {
            double d[3], r2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                d[c] = x_mm[3 * (size_t)j + c] - x_nnp[3 * (size_t)i + c];
                r2 += d[c] * d[c];
            }
            const double r = sqrt(r2);
            if (cutoff > 0.0 && r >= cutoff) continue;
            double v, dv;
            pair_term(k, par_nnp[3 * i], par_mm[3 * (size_t)j], par_nnp[3 * i + 1],
                      par_mm[3 * (size_t)j + 1], par_nnp[3 * i + 2], par_mm[3 * (size_t)j + 2], r,
                      &v, &dv);
            e += v;
            a += fabs(v);
            /* d r / d x_j = d / r, d r / d x_i = -d / r */
            for (int c = 0; c < 3; ++c) {
                const double g = dv * d[c] / r;
                F_mm[3 * (size_t)j + c] -= g;
                F_nnp[3 * (size_t)i + c] += g;
            }
        }
    *E = e;
    if (abs_sum) *abs_sum = a;
}
