/*
 * nnp_oracle.c -- plain, slow FP64 CPU oracle for the NNP energy / force path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this file; it exists so that tests, the smoke check and the CPU baseline
 * of the benchmark can compare the GPU library against an obviously correct
 * implementation.  It shares no code, header or table with the HIP library.
 *
 * What is computed (all in double precision, brute force, no cell lists):
 *
 *   V_NNP(Z, r)            -- Methods, Eq. 2 (the total charge is dropped: the
 *                             ANI-2x family handles neutral molecules only,
 *                             Introduction).
 *   F = -grad V_NNP        -- Methods, Eq. 3, by the exact chain rule.
 *   ensemble average       -- Methods, optimisation paragraph (ANI-2x is an
 *                             ensemble of 8 networks, averaged).
 *
 * The paper names the featuriser only as the modified Behler-Parrinello
 * symmetry functions of ANI with a 5.1 A cutoff over H,C,N,O,F,S,Cl
 * (Introduction; Methods, software stack).  The form written out below is the
 * published ANI form it cites:
 *
 *   cutoff    fc(r) = 0.5 cos(pi r / Rc) + 0.5 for r < Rc, else 0
 *   radial    G_i[nR*s_j + k] += pref_R * exp(-etaR (r_ij - ShfR_k)^2) fc(r_ij; Rcr)
 *             over every j != i with r_ij < Rcr
 *   angular   over every unordered pair {j,k} (j != k, both != i) with
 *             r_ij, r_ik < Rca:
 *               c   = cos(theta_ijk),  c' = s_ang * c,  theta' = arccos(c')
 *               cos(theta' - ShfZ_z) = c' cos ShfZ_z + sqrt(1 - c'^2) sin ShfZ_z
 *               term = 2 ((1 + cos(theta' - ShfZ_z)) / 2)^zeta
 *                        * exp(-etaA ((r_ij + r_ik)/2 - ShfA_a)^2)
 *                        * fc(r_ij; Rca) fc(r_ik; Rca)
 *             added to G_i[S*nR + (nA*nZ) * p(s_j, s_k) + nZ*a + z] where
 *             p(b, c), b <= c, is the row-major index of the upper triangle
 *             of the S x S species-pair matrix.
 *   network   per model m and element s: z_l = W_l a_{l-1} + b_l, a_l = CELU(z_l)
 *             on hidden layers, e = z_L (one output); CELU(z) = z for z >= 0,
 *             alpha (exp(z/alpha) - 1) otherwise.
 *   energy    E_mol = u * ( (1/M) sum_m sum_i e_{m,i} + sum_i SAE[s_i] )
 *
 * Weights are one flat FP64 array, ordered [model][element][layer] and, per
 * layer, W (out x in, row-major) followed by b (out).  Every element may have
 * networks of its own widths (the ANI-2x element networks differ in size);
 * then the (model, element) blocks have different lengths.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

typedef struct {
    int32_t n_species;        /* S */
    int32_t n_shf_r;          /* nR */
    int32_t n_shf_a;          /* nA */
    int32_t n_shf_z;          /* nZ */
    double rcr, rca;          /* cutoffs, Angstrom */
    double eta_r, eta_a, zeta;
    double angle_scale;       /* s_ang, the factor applied to cos(theta) before arccos */
    double radial_pref;       /* pref_R */
    const double* shf_r;      /* [nR] */
    const double* shf_a;      /* [nA] */
    const double* shf_z;      /* [nZ] */
} orc_aev_t;

typedef struct {
    int32_t n_models;         /* M */
    int32_t n_species;        /* S */
    int32_t n_layers;         /* L (number of affine layers) */
    const int32_t* widths;    /* [L+1]; widths[0] = AEV dimension, widths[L] = 1 */
    double celu_alpha;
    const double* weights;    /* packed, see the file header */
    const int32_t* species_widths;   /* [S][L+1] per-element widths, or NULL (all `widths`) */
} orc_net_t;

/* ------------------------------------------------------------------------ */
/* sizes                                                                     */

int32_t orc_aev_dim(const orc_aev_t* p)
{
    int32_t S = p->n_species;
    return S * p->n_shf_r + (S * (S + 1) / 2) * p->n_shf_a * p->n_shf_z;
}

/* the layer widths of element s's networks */
static const int32_t* widths_of(const orc_net_t* n, int s)
{
    return n->species_widths ? n->species_widths + (int64_t)s * (n->n_layers + 1) : n->widths;
}

/* parameters of one network of element s */
static int64_t net_size_of(const orc_net_t* n, int s)
{
    const int32_t* w = widths_of(n, s);
    int64_t sz = 0;
    for (int l = 0; l < n->n_layers; ++l)
        sz += (int64_t)w[l + 1] * w[l] + w[l + 1];
    return sz;
}

/* parameters of one model (all its element networks) */
int64_t orc_net_size(const orc_net_t* n)
{
    int64_t sz = 0;
    for (int s = 0; s < n->n_species; ++s) sz += net_size_of(n, s);
    return sz;
}

int64_t orc_weights_size(const orc_net_t* n)
{
    return (int64_t)n->n_models * orc_net_size(n);
}

/* offset of network (m, s) in the packed array */
static int64_t net_offset(const orc_net_t* n, int m, int s)
{
    int64_t off = (int64_t)m * orc_net_size(n);
    for (int t = 0; t < s; ++t) off += net_size_of(n, t);
    return off;
}

static const double* net_ptr(const orc_net_t* n, int m, int s)
{
    return n->weights + net_offset(n, m, s);
}

/* ------------------------------------------------------------------------ */
/* cutoff function and its derivative                                        */

double orc_fc(double r, double rc)
{
    if (r >= rc) return 0.0;
    return 0.5 * cos(ORC_PI * r / rc) + 0.5;
}

double orc_dfc(double r, double rc)
{
    if (r >= rc) return 0.0;
    return -0.5 * ORC_PI / rc * sin(ORC_PI * r / rc);
}

/* upper-triangle index of the unordered element pair (b, c) */
static int pair_index(int b, int c, int S)
{
    if (b > c) { int t = b; b = c; c = t; }
    return b * S - b * (b - 1) / 2 + (c - b);
}

static double dist(const double* x, int i, int j, double u[3])
{
    double d0 = x[3 * j + 0] - x[3 * i + 0];
    double d1 = x[3 * j + 1] - x[3 * i + 1];
    double d2 = x[3 * j + 2] - x[3 * i + 2];
    double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    u[0] = d0 / r; u[1] = d1 / r; u[2] = d2 / r;
    return r;
}

/* ------------------------------------------------------------------------ */
/* The per-term values and partial derivatives.  One radial term depends on   */
/* r_ij only; one angular term on (r_ij, r_ik, c).                            */

static void radial_term(const orc_aev_t* p, int k, double r, double* val, double* d_dr)
{
    double dr = r - p->shf_r[k];
    double g = p->radial_pref * exp(-p->eta_r * dr * dr);
    double fc = orc_fc(r, p->rcr), dfc = orc_dfc(r, p->rcr);
    *val = g * fc;
    *d_dr = g * (-2.0 * p->eta_r * dr * fc + dfc);
}

/* angular factor (includes the leading 2) and its derivative in c */
static void angle_factor(const orc_aev_t* p, int z, double c, double* val, double* d_dc)
{
    double cp = p->angle_scale * c;
    double sn = sqrt(1.0 - cp * cp);
    double cs = cos(p->shf_z[z]), ss = sin(p->shf_z[z]);
    double cz = cp * cs + sn * ss;                 /* cos(theta' - ShfZ) */
    double half = 0.5 * (1.0 + cz);
    *val = 2.0 * pow(half, p->zeta);
    double dcz_dc = p->angle_scale * (cs - cp * ss / sn);
    *d_dc = (p->zeta == 0.0) ? 0.0 : 2.0 * p->zeta * pow(half, p->zeta - 1.0) * 0.5 * dcz_dc;
}

/* radial-distance factor of the angular term and its derivative in rmean */
static void dist_factor(const orc_aev_t* p, int a, double rm, double* val, double* d_drm)
{
    double d = rm - p->shf_a[a];
    double g = exp(-p->eta_a * d * d);
    *val = g;
    *d_drm = -2.0 * p->eta_a * d * g;
}

/* ------------------------------------------------------------------------ */
/* AEV of one molecule                                                         */

void orc_aev(const orc_aev_t* p, int32_t n, const int32_t* species, const double* x,
             double* aev)
{
    const int S = p->n_species, nR = p->n_shf_r, nA = p->n_shf_a, nZ = p->n_shf_z;
    const int D = orc_aev_dim(p);
    const int rad = S * nR;
    memset(aev, 0, sizeof(double) * (size_t)n * D);
    for (int i = 0; i < n; ++i) {
        double* G = aev + (size_t)i * D;
        /* radial: every ordered neighbour j of i */
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double u[3];
            double r = dist(x, i, j, u);
            if (r >= p->rcr) continue;
            for (int k = 0; k < nR; ++k) {
                double v, dv;
                radial_term(p, k, r, &v, &dv);
                G[nR * species[j] + k] += v;
            }
        }
        /* angular: every unordered pair {j, k} */
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double uj[3];
            double rj = dist(x, i, j, uj);
            if (rj >= p->rca) continue;
            for (int k = j + 1; k < n; ++k) {
                if (k == i) continue;
                double uk[3];
                double rk = dist(x, i, k, uk);
                if (rk >= p->rca) continue;
                double c = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
                double fcc = orc_fc(rj, p->rca) * orc_fc(rk, p->rca);
                int base = rad + nA * nZ * pair_index(species[j], species[k], S);
                for (int a = 0; a < nA; ++a) {
                    double fa, dfa;
                    dist_factor(p, a, 0.5 * (rj + rk), &fa, &dfa);
                    for (int z = 0; z < nZ; ++z) {
                        double fz, dfz;
                        angle_factor(p, z, c, &fz, &dfz);
                        G[base + nZ * a + z] += fz * fa * fcc;
                    }
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Vector-Jacobian product: gx[j] = sum_i sum_slot gG[i][slot] dG_i[slot]/dx_j */
/* (gx is overwritten; it is dE/dx when gG = dE/dG).                          */

void orc_aev_vjp(const orc_aev_t* p, int32_t n, const int32_t* species, const double* x,
                 const double* gG, double* gx)
{
    const int S = p->n_species, nR = p->n_shf_r, nA = p->n_shf_a, nZ = p->n_shf_z;
    const int D = orc_aev_dim(p);
    const int rad = S * nR;
    memset(gx, 0, sizeof(double) * 3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const double* g = gG + (size_t)i * D;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double u[3];
            double r = dist(x, i, j, u);
            if (r >= p->rcr) continue;
            double dE_dr = 0.0;
            for (int k = 0; k < nR; ++k) {
                double v, dv;
                radial_term(p, k, r, &v, &dv);
                dE_dr += g[nR * species[j] + k] * dv;
            }
            /* dr_ij/dx_j = u_ij, dr_ij/dx_i = -u_ij */
            for (int d = 0; d < 3; ++d) {
                gx[3 * j + d] += dE_dr * u[d];
                gx[3 * i + d] -= dE_dr * u[d];
            }
        }
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double uj[3];
            double rj = dist(x, i, j, uj);
            if (rj >= p->rca) continue;
            for (int k = j + 1; k < n; ++k) {
                if (k == i) continue;
                double uk[3];
                double rk = dist(x, i, k, uk);
                if (rk >= p->rca) continue;
                double c = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
                double fcj = orc_fc(rj, p->rca), fck = orc_fc(rk, p->rca);
                double dfcj = orc_dfc(rj, p->rca), dfck = orc_dfc(rk, p->rca);
                double fcc = fcj * fck;
                int base = rad + nA * nZ * pair_index(species[j], species[k], S);
                double D_c = 0.0, D_rj = 0.0, D_rk = 0.0;
                for (int a = 0; a < nA; ++a) {
                    double fa, dfa;
                    dist_factor(p, a, 0.5 * (rj + rk), &fa, &dfa);
                    for (int z = 0; z < nZ; ++z) {
                        double fz, dfz;
                        angle_factor(p, z, c, &fz, &dfz);
                        double w = g[base + nZ * a + z];
                        D_c += w * dfz * fa * fcc;
                        /* d(term)/dr_ij: the rmean factor moves with half of dr_ij */
                        D_rj += w * fz * (0.5 * dfa * fcc + fa * dfcj * fck);
                        D_rk += w * fz * (0.5 * dfa * fcc + fa * fcj * dfck);
                    }
                }
                for (int d = 0; d < 3; ++d) {
                    double dc_dxj = (uk[d] - c * uj[d]) / rj;
                    double dc_dxk = (uj[d] - c * uk[d]) / rk;
                    double gj = D_rj * uj[d] + D_c * dc_dxj;
                    double gk = D_rk * uk[d] + D_c * dc_dxk;
                    gx[3 * j + d] += gj;
                    gx[3 * k + d] += gk;
                    gx[3 * i + d] -= gj + gk;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Jacobian-vector product: gdot[i][slot] = sum_j dG_i[slot]/dx_j . v_j      */

void orc_aev_jvp(const orc_aev_t* p, int32_t n, const int32_t* species, const double* x,
                 const double* v, double* gdot)
{
    const int S = p->n_species, nR = p->n_shf_r, nA = p->n_shf_a, nZ = p->n_shf_z;
    const int D = orc_aev_dim(p);
    const int rad = S * nR;
    memset(gdot, 0, sizeof(double) * (size_t)n * D);
    for (int i = 0; i < n; ++i) {
        double* G = gdot + (size_t)i * D;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double u[3];
            double r = dist(x, i, j, u);
            if (r >= p->rcr) continue;
            double rdot = 0.0;
            for (int d = 0; d < 3; ++d) rdot += u[d] * (v[3 * j + d] - v[3 * i + d]);
            for (int k = 0; k < nR; ++k) {
                double val, dv;
                radial_term(p, k, r, &val, &dv);
                G[nR * species[j] + k] += dv * rdot;
            }
        }
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double uj[3];
            double rj = dist(x, i, j, uj);
            if (rj >= p->rca) continue;
            for (int k = j + 1; k < n; ++k) {
                if (k == i) continue;
                double uk[3];
                double rk = dist(x, i, k, uk);
                if (rk >= p->rca) continue;
                double c = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
                double fcj = orc_fc(rj, p->rca), fck = orc_fc(rk, p->rca);
                double dfcj = orc_dfc(rj, p->rca), dfck = orc_dfc(rk, p->rca);
                double fcc = fcj * fck;
                double rjdot = 0.0, rkdot = 0.0, cdot = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double vij = v[3 * j + d] - v[3 * i + d];
                    double vik = v[3 * k + d] - v[3 * i + d];
                    rjdot += uj[d] * vij;
                    rkdot += uk[d] * vik;
                    /* dc/dx_j . v_j + dc/dx_k . v_k + dc/dx_i . v_i */
                    cdot += (uk[d] - c * uj[d]) / rj * vij + (uj[d] - c * uk[d]) / rk * vik;
                }
                int base = rad + nA * nZ * pair_index(species[j], species[k], S);
                for (int a = 0; a < nA; ++a) {
                    double fa, dfa;
                    dist_factor(p, a, 0.5 * (rj + rk), &fa, &dfa);
                    for (int z = 0; z < nZ; ++z) {
                        double fz, dfz;
                        angle_factor(p, z, c, &fz, &dfz);
                        double d_rj = fz * (0.5 * dfa * fcc + fa * dfcj * fck);
                        double d_rk = fz * (0.5 * dfa * fcc + fa * fcj * dfck);
                        double d_c = dfz * fa * fcc;
                        G[base + nZ * a + z] += d_rj * rjdot + d_rk * rkdot + d_c * cdot;
                    }
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Atomic network                                                             */

static double celu(double z, double al) { return z >= 0.0 ? z : al * (exp(z / al) - 1.0); }
static double celu_d1(double z, double al) { return z >= 0.0 ? 1.0 : exp(z / al); }
static double celu_d2(double z, double al) { return z >= 0.0 ? 0.0 : exp(z / al) / al; }

static int max_width(const orc_net_t* n, int s)
{
    const int32_t* wd = widths_of(n, s);
    int w = 0;
    for (int l = 0; l <= n->n_layers; ++l) if (wd[l] > w) w = wd[l];
    return w;
}

/*
 * One atom, one model: e = NN_{m,s}(G).  If dG != NULL, also dG = de/dG.
 * Returns e.
 */
double orc_atomic_nn(const orc_net_t* n, int32_t m, int32_t s, const double* G, double* dG)
{
    const int L = n->n_layers, W = max_width(n, s);
    const int32_t* wd = widths_of(n, s);
    const double al = n->celu_alpha;
    double* z = (double*)calloc((size_t)L * W, sizeof(double));  /* pre-activations */
    double* a = (double*)calloc((size_t)(L + 1) * W, sizeof(double));
    memcpy(a, G, sizeof(double) * wd[0]);
    const double* wp = net_ptr(n, m, s);
    const double* Wl[64];
    const double* bl[64];
    for (int l = 0; l < L; ++l) {
        int nin = wd[l], nout = wd[l + 1];
        Wl[l] = wp; bl[l] = wp + (int64_t)nout * nin;
        wp += (int64_t)nout * nin + nout;
        for (int o = 0; o < nout; ++o) {
            double acc = bl[l][o];
            for (int k = 0; k < nin; ++k) acc += Wl[l][(int64_t)o * nin + k] * a[l * W + k];
            z[l * W + o] = acc;
            a[(l + 1) * W + o] = (l + 1 < L) ? celu(acc, al) : acc;
        }
    }
    double e = a[L * W + 0];
    if (dG) {
        /* reverse: adjoint of the output is 1 */
        double* g = (double*)calloc((size_t)W, sizeof(double));
        double* gp = (double*)calloc((size_t)W, sizeof(double));
        g[0] = 1.0;
        for (int l = L - 1; l >= 0; --l) {
            int nin = wd[l], nout = wd[l + 1];
            /* g holds dE/dz_l (for l = L-1 the output is linear) */
            memset(gp, 0, sizeof(double) * W);
            for (int o = 0; o < nout; ++o)
                for (int k = 0; k < nin; ++k) gp[k] += Wl[l][(int64_t)o * nin + k] * g[o];
            if (l > 0)
                for (int k = 0; k < nin; ++k) g[k] = gp[k] * celu_d1(z[(l - 1) * W + k], al);
            else
                memcpy(dG, gp, sizeof(double) * nin);
        }
        free(g); free(gp);
    }
    free(z); free(a);
    return e;
}

/*
 * One atom, one model: accumulate into gw (packed like the weights of this
 * (m, s) network) the parameter gradient of  alpha * e + beta * edot, where
 * edot is the tangent of e along the AEV tangent Gdot.
 */
static void atomic_nn_param_grad(const orc_net_t* n, int32_t m, int32_t s, const double* G,
                                 const double* Gdot, double alpha, double beta, double* gw)
{
    const int L = n->n_layers, W = max_width(n, s);
    const int32_t* wd = widths_of(n, s);
    const double al = n->celu_alpha;
    double* z = (double*)calloc((size_t)L * W, sizeof(double));
    double* zd = (double*)calloc((size_t)L * W, sizeof(double));
    double* a = (double*)calloc((size_t)(L + 1) * W, sizeof(double));
    double* ad = (double*)calloc((size_t)(L + 1) * W, sizeof(double));
    memcpy(a, G, sizeof(double) * wd[0]);
    memcpy(ad, Gdot, sizeof(double) * wd[0]);
    const double* wp = net_ptr(n, m, s);
    const double* Wl[64];
    int64_t off[64];
    int64_t o0 = 0;
    for (int l = 0; l < L; ++l) {
        int nin = wd[l], nout = wd[l + 1];
        Wl[l] = wp + o0; off[l] = o0;
        const double* b = Wl[l] + (int64_t)nout * nin;
        o0 += (int64_t)nout * nin + nout;
        for (int o = 0; o < nout; ++o) {
            double acc = b[o], accd = 0.0;
            for (int k = 0; k < nin; ++k) {
                acc += Wl[l][(int64_t)o * nin + k] * a[l * W + k];
                accd += Wl[l][(int64_t)o * nin + k] * ad[l * W + k];
            }
            z[l * W + o] = acc;
            zd[l * W + o] = accd;
            if (l + 1 < L) {
                a[(l + 1) * W + o] = celu(acc, al);
                ad[(l + 1) * W + o] = celu_d1(acc, al) * accd;
            } else {
                a[(l + 1) * W + o] = acc;
                ad[(l + 1) * W + o] = accd;
            }
        }
    }
    /* reverse through both the primal and the tangent graph */
    double* zb = (double*)calloc((size_t)W, sizeof(double));   /* adjoint of z_l    */
    double* zdb = (double*)calloc((size_t)W, sizeof(double));  /* adjoint of zdot_l */
    double* ab = (double*)calloc((size_t)W, sizeof(double));   /* adjoint of a_l    */
    double* adb = (double*)calloc((size_t)W, sizeof(double));  /* adjoint of adot_l */
    zb[0] = alpha;
    zdb[0] = beta;
    for (int l = L - 1; l >= 0; --l) {
        int nin = wd[l], nout = wd[l + 1];
        double* gW = gw + off[l];
        double* gb = gW + (int64_t)nout * nin;
        for (int o = 0; o < nout; ++o) {
            gb[o] += zb[o];
            for (int k = 0; k < nin; ++k)
                gW[(int64_t)o * nin + k] += zb[o] * a[l * W + k] + zdb[o] * ad[l * W + k];
        }
        if (l == 0) break;
        memset(ab, 0, sizeof(double) * W);
        memset(adb, 0, sizeof(double) * W);
        for (int o = 0; o < nout; ++o)
            for (int k = 0; k < nin; ++k) {
                ab[k] += Wl[l][(int64_t)o * nin + k] * zb[o];
                adb[k] += Wl[l][(int64_t)o * nin + k] * zdb[o];
            }
        /* a = celu(z), adot = celu'(z) zdot */
        for (int k = 0; k < nin; ++k) {
            double zz = z[(l - 1) * W + k];
            zb[k] = ab[k] * celu_d1(zz, al) + adb[k] * celu_d2(zz, al) * zd[(l - 1) * W + k];
            zdb[k] = adb[k] * celu_d1(zz, al);
        }
    }
    free(z); free(zd); free(a); free(ad); free(zb); free(zdb); free(ab); free(adb);
}

/* ------------------------------------------------------------------------ */
/* Batched energy and forces                                                  */

/*
 * n_mols molecules in CSR form (mol_off[n_mols+1] into the atom arrays).
 * E[n_mols] in units of energy_scale * (network output), F[n_atoms*3] = -dE/dx.
 * sae may be NULL (all zero).  Molecules are independent (OpenMP over them;
 * the network part runs over atoms).
 */
void orc_energy_forces(const orc_aev_t* p, const orc_net_t* net, double energy_scale,
                       const double* sae, int32_t n_mols, const int32_t* mol_off,
                       const int32_t* species, const double* x, double* E, double* F)
{
    const int D = orc_aev_dim(p);
    const int32_t A = mol_off[n_mols];
    const int M = net->n_models;
    double* G = (double*)malloc(sizeof(double) * (size_t)A * D + 8);
    double* gG = (double*)malloc(sizeof(double) * (size_t)A * D + 8);
    double* eat = (double*)malloc(sizeof(double) * (size_t)A + 8);

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < n_mols; ++b) {
        int a0 = mol_off[b], n = mol_off[b + 1] - a0;
        if (n > 0) orc_aev(p, n, species + a0, x + 3 * (size_t)a0, G + (size_t)a0 * D);
    }

#pragma omp parallel
    {
        double* dg = (double*)malloc(sizeof(double) * (size_t)D);
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < A; ++i) {
            double e = 0.0;
            double* gi = gG + (size_t)i * D;
            memset(gi, 0, sizeof(double) * D);
            for (int m = 0; m < M; ++m) {
                e += orc_atomic_nn(net, m, species[i], G + (size_t)i * D, dg);
                for (int k = 0; k < D; ++k) gi[k] += dg[k];
            }
            /* dE/dG_i = (u / M) sum_m de_m/dG_i */
            for (int k = 0; k < D; ++k) gi[k] *= energy_scale / M;
            eat[i] = energy_scale * (e / M + (sae ? sae[species[i]] : 0.0));
        }
        free(dg);
    }

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < n_mols; ++b) {
        int a0 = mol_off[b], n = mol_off[b + 1] - a0;
        double acc = 0.0;
        for (int i = a0; i < a0 + n; ++i) acc += eat[i];
        E[b] = acc;
        if (n > 0) {
            orc_aev_vjp(p, n, species + a0, x + 3 * (size_t)a0, gG + (size_t)a0 * D,
                        F + 3 * (size_t)a0);
            for (int k = 0; k < 3 * n; ++k) F[3 * (size_t)a0 + k] = -F[3 * (size_t)a0 + k];
        }
    }
    free(G); free(gG); free(eat);
}

/*
 * Parameter gradient of a loss L(E, F) given its cotangents gE = dL/dE [n_mols]
 * and gF = dL/dF [n_atoms*3]:
 *
 *   dL/dW = sum_b gE_b dE_b/dW + sum_{i,c} gF_ic dF_ic/dW
 *
 * F = -dE/dx, so the second sum is -d/dW of sum_i (dE/dG_i . Gdot_i) with
 * Gdot = (dG/dx) gF, the AEV tangent along gF (independent of W); per atom and
 * model that inner product is (u/M) times the tangent edot of the network
 * output along Gdot_i.  gw is overwritten, packed like the weights.
 */
void orc_param_grad(const orc_aev_t* p, const orc_net_t* net, double energy_scale,
                    int32_t n_mols, const int32_t* mol_off, const int32_t* species,
                    const double* x, const double* gE, const double* gF, double* gw)
{
    const int D = orc_aev_dim(p);
    const int32_t A = mol_off[n_mols];
    const int M = net->n_models, S = net->n_species;
    double* G = (double*)malloc(sizeof(double) * (size_t)A * D + 8);
    double* Gd = (double*)malloc(sizeof(double) * (size_t)A * D + 8);
    int32_t* mol_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)A + 8);

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < n_mols; ++b) {
        int a0 = mol_off[b], n = mol_off[b + 1] - a0;
        for (int i = a0; i < a0 + n; ++i) mol_of[i] = b;
        if (n == 0) continue;
        orc_aev(p, n, species + a0, x + 3 * (size_t)a0, G + (size_t)a0 * D);
        orc_aev_jvp(p, n, species + a0, x + 3 * (size_t)a0, gF + 3 * (size_t)a0,
                    Gd + (size_t)a0 * D);
    }

    memset(gw, 0, sizeof(double) * (size_t)orc_weights_size(net));
    /* one (model, element) network per task, atoms in order: deterministic */
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int m = 0; m < M; ++m)
        for (int s = 0; s < S; ++s) {
            double* g = gw + net_offset(net, m, s);
            for (int i = 0; i < A; ++i) {
                if (species[i] != s) continue;
                double alpha = energy_scale / M * gE[mol_of[i]];
                double beta = -energy_scale / M;
                atomic_nn_param_grad(net, m, s, G + (size_t)i * D, Gd + (size_t)i * D, alpha,
                                     beta, g);
            }
        }
    free(G); free(Gd); free(mol_of);
}

/* number of OpenMP threads the oracle will use (reported with timings) */
int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
