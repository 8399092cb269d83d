/*
 * chem_oracle.c -- plain, slow, table-driven FP64 CPU oracle for per-cell
 * chemistry integration.  TEST INFRASTRUCTURE ONLY: it exists so that the GPU
 * path can be checked against something written directly from the paper.  It
 * shares no code, header or table with the GPU library and must never be
 * linked into it.
 *
 * What it computes (paper: Sec. 2.1.2 and Sec. 2.2.3):
 *   - NASA 7-coefficient thermodynamics per species (Eq. 10's h_i, c_pi);
 *   - mass-action molar production rates (Eq. 15-16), forward rate in
 *     Arrhenius form, reverse rate from the equilibrium constant, and a
 *     third-body concentration multiplying both directions when a reaction
 *     lists collision efficiencies;
 *   - the chemistry ODE of Eq. 20 with the species source of Eq. 14, written
 *     for u = (T, Y_1..Y_N) at constant density and internal energy
 *     (constant-volume adiabatic closure for dT/dt);
 *   - one step of the two-register low-storage RK (Eq. 21) with the embedded
 *     error register, and the WRMS step-size controller of Eq. 22;
 *   - a per-cell driver over one flow time step;
 *   - for comparison, a full-storage Runge-Kutta-Fehlberg 4(5) step under the
 *     same controller (exponent 1/5 for its fourth-order error estimate);
 *   - and, as the implicit comparator the paper measures against, a
 *     linearly implicit Rosenbrock step: fourth order with an embedded third
 *     order solution (Shampine's parameter set in the Kaps-Rentrop form),
 *     the exact Jacobian by complex-step differentiation of the RHS, a dense
 *     LU factorisation with partial pivoting, the same controller
 *     (exponent 1/4).
 *
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes of the repository):
 *   - scheme coefficients: Kennedy-Carpenter-Lewis RK4(3)5[2R+]C (the paper's
 *     "fourth-order, five-stage, low-storage embedded" scheme, its ref. [37]);
 *   - Eq. 22's h_min/h_max clamp is applied to the step factor: [0.2, 5];
 *     exponent 1/4; the WRMS weights use |u| at the start of the step; the
 *     mean runs over all N+1 components;
 *   - accept iff err <= 1; NaN error => reject with factor 0.2; err == 0 =>
 *     factor 5; the final step is clipped to end exactly at dt;
 *   - NASA-7 range: T < Tmid uses the low range; no clamping outside the fit;
 *   - the equilibrium constant uses the standard pressure given in the
 *     mechanism file (1 atm) and R in cgs units.
 *
 * Units: cgs (mol/cm^3, g/cm^3, s); activation energy in J/mol.
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared -o liboracle.so chem_oracle.c -lm
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_R_J 8.31446261815324       /* J/(mol K) */
#define OR_R_CGS 8.31446261815324e7   /* erg/(mol K) */

enum { OR_OK = 0, OR_MAXSTEPS = 1, OR_NONFINITE = 2, OR_H_UNDERFLOW = 3 };

typedef struct {
    int n_reac, n_prod;
    int reac_sp[8], reac_nu[8];
    int prod_sp[8], prod_nu[8];
    double A, b, Ea;
    int third_body;
    double *eff; /* [ns] */
} or_reaction;

typedef struct {
    int ne, ns, nr;
    double pstd;
    double *ew;      /* [ne] element atomic weights */
    char (*sp_name)[32];
    double *W;       /* [ns] */
    int *comp;       /* [ns*ne] */
    double *Tmid;    /* [ns] */
    double *lo;      /* [ns*7] */
    double *hi;      /* [ns*7] */
    or_reaction *rx; /* [nr] */
} or_mech;

/* ------------------------------------------------------------------ parser */
static char *next_tok(char **p) {
    char *s = *p;
    while (*s == ' ' || *s == '\t') s++;
    if (*s == 0 || *s == '\n') { *p = s; return NULL; }
    char *t = s;
    while (*s && *s != ' ' && *s != '\t' && *s != '\n') s++;
    if (*s) { *s = 0; s++; }
    *p = s;
    return t;
}

static int read_line(FILE *f, char *buf, int len) {
    for (;;) {
        if (!fgets(buf, len, f)) return 0;
        char *s = buf;
        while (*s == ' ' || *s == '\t') s++;
        if (*s == '#' || *s == '\n' || *s == 0) continue;
        return 1;
    }
}

static int species_index(const or_mech *m, const char *name) {
    for (int k = 0; k < m->ns; k++)
        if (strcmp(m->sp_name[k], name) == 0) return k;
    return -1;
}

void or_mech_free(or_mech *m) {
    if (!m) return;
    if (m->rx)
        for (int j = 0; j < m->nr; j++) free(m->rx[j].eff);
    free(m->rx); free(m->sp_name); free(m->W); free(m->comp); free(m->ew);
    free(m->Tmid); free(m->lo); free(m->hi); free(m);
}

/* Returns 0 on success, else the (1-based) offending line-count; *out set on success. */
int or_mech_load(const char *path, or_mech **out) {
    FILE *f = fopen(path, "r");
    if (!f) return -1;
    char buf[65536];
    int line = 0;
    or_mech *m = calloc(1, sizeof(or_mech));
#define FAIL() do { fclose(f); or_mech_free(m); return line > 0 ? line : 1; } while (0)
    char *p, *t;
    if (!read_line(f, buf, sizeof buf) || strncmp(buf, "MECH 1", 6) != 0) FAIL();
    line++;
    for (;;) {
        if (!read_line(f, buf, sizeof buf)) FAIL();
        line++;
        p = buf;
        t = next_tok(&p);
        if (!t) FAIL();
        if (strcmp(t, "name") == 0) continue;
        if (strcmp(t, "pstd") == 0) { m->pstd = strtod(next_tok(&p), NULL); continue; }
        if (strcmp(t, "elements") == 0) {
            m->ne = atoi(next_tok(&p));
            m->ew = calloc(m->ne > 0 ? m->ne : 1, sizeof(double));
            for (int e = 0; e < m->ne; e++) {
                if (!read_line(f, buf, sizeof buf)) FAIL();
                line++;
                p = buf;
                t = next_tok(&p); if (!t) FAIL();
                t = next_tok(&p); if (!t) FAIL();
                m->ew[e] = strtod(t, NULL);
            }
            continue;
        }
        if (strcmp(t, "species") == 0) {
            m->ns = atoi(next_tok(&p));
            int ns = m->ns;
            m->sp_name = calloc(ns, 32);
            m->W = calloc(ns, sizeof(double));
            m->comp = calloc((size_t)ns * (m->ne > 0 ? m->ne : 1), sizeof(int));
            m->Tmid = calloc(ns, sizeof(double));
            m->lo = calloc((size_t)ns * 7, sizeof(double));
            m->hi = calloc((size_t)ns * 7, sizeof(double));
            for (int k = 0; k < ns; k++) {
                if (!read_line(f, buf, sizeof buf)) FAIL();
                line++;
                p = buf;
                t = next_tok(&p); if (!t) FAIL();
                strncpy(m->sp_name[k], t, 31);
                t = next_tok(&p); if (!t) FAIL(); m->W[k] = strtod(t, NULL);
                for (int e = 0; e < m->ne; e++) { t = next_tok(&p); if (!t) FAIL(); m->comp[k * m->ne + e] = atoi(t); }
                t = next_tok(&p); if (!t) FAIL();                         /* Tlow */
                t = next_tok(&p); if (!t) FAIL(); m->Tmid[k] = strtod(t, NULL);
                t = next_tok(&p); if (!t) FAIL();                         /* Thigh */
                for (int i = 0; i < 7; i++) { t = next_tok(&p); if (!t) FAIL(); m->lo[k * 7 + i] = strtod(t, NULL); }
                for (int i = 0; i < 7; i++) { t = next_tok(&p); if (!t) FAIL(); m->hi[k * 7 + i] = strtod(t, NULL); }
            }
            continue;
        }
        if (strcmp(t, "reactions") == 0) {
            m->nr = atoi(next_tok(&p));
            m->rx = calloc(m->nr, sizeof(or_reaction));
            for (int j = 0; j < m->nr; j++) {
                or_reaction *r = &m->rx[j];
                if (!read_line(f, buf, sizeof buf)) FAIL();
                line++;
                p = buf;
                t = next_tok(&p); if (!t || strcmp(t, "reaction") != 0) FAIL();
                r->A = strtod(next_tok(&p), NULL);
                r->b = strtod(next_tok(&p), NULL);
                r->Ea = strtod(next_tok(&p), NULL);
                r->third_body = atoi(next_tok(&p));
                for (int side = 0; side < 2; side++) {
                    if (!read_line(f, buf, sizeof buf)) FAIL();
                    line++;
                    p = buf;
                    t = next_tok(&p);
                    if (!t || strcmp(t, side == 0 ? "reactants" : "products") != 0) FAIL();
                    int n = atoi(next_tok(&p));
                    if (n < 1 || n > 8) FAIL();
                    for (int i = 0; i < n; i++) {
                        char *nm = next_tok(&p);
                        char *nu = next_tok(&p);
                        if (!nm || !nu) FAIL();
                        int k = species_index(m, nm);
                        if (k < 0) FAIL();
                        if (side == 0) { r->reac_sp[i] = k; r->reac_nu[i] = atoi(nu); }
                        else { r->prod_sp[i] = k; r->prod_nu[i] = atoi(nu); }
                    }
                    if (side == 0) r->n_reac = n; else r->n_prod = n;
                }
                if (r->third_body) {
                    if (!read_line(f, buf, sizeof buf)) FAIL();
                    line++;
                    p = buf;
                    t = next_tok(&p); if (!t || strcmp(t, "efficiencies") != 0) FAIL();
                    r->eff = calloc(m->ns, sizeof(double));
                    for (int k = 0; k < m->ns; k++) { t = next_tok(&p); if (!t) FAIL(); r->eff[k] = strtod(t, NULL); }
                }
            }
            continue;
        }
        if (strcmp(t, "end") == 0) break;
        FAIL();
    }
#undef FAIL
    fclose(f);
    *out = m;
    return 0;
}

void or_mech_dims(const or_mech *m, int *ne, int *ns, int *nr) {
    *ne = m->ne; *ns = m->ns; *nr = m->nr;
}

void or_mech_elements(const or_mech *m, double *ew) {
    for (int e = 0; e < m->ne; e++) ew[e] = m->ew[e];
}

void or_mech_species(const or_mech *m, double *W, int *comp) {
    for (int k = 0; k < m->ns; k++) {
        W[k] = m->W[k];
        for (int e = 0; e < m->ne; e++) comp[k * m->ne + e] = m->comp[k * m->ne + e];
    }
}

/* Net stoichiometric matrix nu[j*ns + k] = nu''_jk - nu'_jk. */
void or_mech_stoich(const or_mech *m, double *nu) {
    memset(nu, 0, sizeof(double) * (size_t)m->nr * m->ns);
    for (int j = 0; j < m->nr; j++) {
        const or_reaction *r = &m->rx[j];
        for (int i = 0; i < r->n_reac; i++) nu[j * m->ns + r->reac_sp[i]] -= r->reac_nu[i];
        for (int i = 0; i < r->n_prod; i++) nu[j * m->ns + r->prod_sp[i]] += r->prod_nu[i];
    }
}

/* ------------------------------------------------------------------ thermo */
/* NASA-7 (Eq. 10's fits): cp/R, h/(RT), s/R for every species at T. */
void or_thermo(const or_mech *m, double T, double *cp_R, double *h_RT, double *s_R) {
    for (int k = 0; k < m->ns; k++) {
        const double *a = (T < m->Tmid[k]) ? &m->lo[k * 7] : &m->hi[k * 7];
        cp_R[k] = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        h_RT[k] = a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
                + a[4] * T * T * T * T / 5.0 + a[5] / T;
        s_R[k] = a[0] * log(T) + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0
               + a[4] * T * T * T * T / 4.0 + a[6];
    }
}

/* ------------------------------------------------- last-bit perturbations */
/* Off (0) by default.  The test suite switches these on to measure how far
 * two correct FP64 integrations of one cell can end apart when they differ
 * only in the last bit of intermediate results, the way any two
 * implementations do (the bound the GPU parity tests use for cells whose
 * accept/reject sequence flips).  Each bit changes one rounding, not the
 * formula:
 *   1  k_f one ulp up (nextafter towards +inf);
 *   2  the step factor's err^(-1/4) taken as 1/sqrt(sqrt(err));
 *   4  wdot accumulated over the reactions in reverse order;
 *   8  k_r from one exponential, exp(ln k_f + dG - dnu ln(pstd/RT)), instead
 *      of k_f / (exp(-dG) (pstd/RT)^dnu).
 * Process-wide; set it only while no integration is running. */
static int or_perturb = 0;

void or_set_perturbation(int mode) { or_perturb = mode; }

/* ------------------------------------------------------------------- rates */
/* Eq. 16 and the Arrhenius / equilibrium-constant rates.  u = (T, Y_1..Y_N).
 * Outputs per reaction (kf, kr, q) and per species wdot [mol/(cm^3 s)]; any
 * output pointer may be NULL. */
void or_rates(const or_mech *m, double rho, const double *u,
              double *kf_out, double *kr_out, double *q_out, double *wdot) {
    int ns = m->ns;
    double T = u[0];
    double *cp = malloc(sizeof(double) * ns), *h = malloc(sizeof(double) * ns);
    double *s = malloc(sizeof(double) * ns), *c = malloc(sizeof(double) * ns);
    or_thermo(m, T, cp, h, s);
    for (int k = 0; k < ns; k++) c[k] = rho * u[1 + k] / m->W[k];
    if (wdot) for (int k = 0; k < ns; k++) wdot[k] = 0.0;
    for (int jj = 0; jj < m->nr; jj++) {
        const int j = (or_perturb & 4) ? m->nr - 1 - jj : jj;
        const or_reaction *r = &m->rx[j];
        double kf = r->A * pow(T, r->b) * exp(-r->Ea / (OR_R_J * T));
        if (or_perturb & 1) kf = nextafter(kf, INFINITY);
        /* Kc = exp(-sum_k nu_jk g_k/RT) * (pstd/(R T))^(sum_k nu_jk) */
        double dG = 0.0;
        int dnu = 0;
        for (int i = 0; i < r->n_prod; i++) {
            int k = r->prod_sp[i];
            dG += r->prod_nu[i] * (h[k] - s[k]);
            dnu += r->prod_nu[i];
        }
        for (int i = 0; i < r->n_reac; i++) {
            int k = r->reac_sp[i];
            dG -= r->reac_nu[i] * (h[k] - s[k]);
            dnu -= r->reac_nu[i];
        }
        double Kc = exp(-dG) * pow(m->pstd / (OR_R_CGS * T), (double)dnu);
        double kr = kf / Kc;
        if (or_perturb & 8) kr = exp(log(kf) + dG - dnu * log(m->pstd / (OR_R_CGS * T)));
        double fwd = kf, rev = kr;
        for (int i = 0; i < r->n_reac; i++)
            for (int n = 0; n < r->reac_nu[i]; n++) fwd *= c[r->reac_sp[i]];
        for (int i = 0; i < r->n_prod; i++)
            for (int n = 0; n < r->prod_nu[i]; n++) rev *= c[r->prod_sp[i]];
        double M = 1.0;
        if (r->third_body) {
            M = 0.0;
            for (int k = 0; k < ns; k++) M += r->eff[k] * c[k];
        }
        double q = M * (fwd - rev);
        if (kf_out) kf_out[j] = kf;
        if (kr_out) kr_out[j] = kr;
        if (q_out) q_out[j] = q;
        if (wdot) {
            for (int i = 0; i < r->n_reac; i++) wdot[r->reac_sp[i]] -= r->reac_nu[i] * q;
            for (int i = 0; i < r->n_prod; i++) wdot[r->prod_sp[i]] += r->prod_nu[i] * q;
        }
    }
    free(cp); free(h); free(s); free(c);
}

/* Right-hand side f(u) of the chemistry ODE (Eq. 14, Eq. 20) for u = (T, Y):
 *   dY_k/dt = W_k wdot_k / rho
 *   dT/dt   = -T * sum_k (h_k/RT - 1) wdot_k / sum_k c_k (cp_k/R - 1)
 * (constant density, constant internal energy). */
void or_rhs(const or_mech *m, double rho, const double *u, double *f) {
    int ns = m->ns;
    double T = u[0];
    double *cp = malloc(sizeof(double) * ns), *h = malloc(sizeof(double) * ns);
    double *s = malloc(sizeof(double) * ns), *w = malloc(sizeof(double) * ns);
    or_thermo(m, T, cp, h, s);
    or_rates(m, rho, u, NULL, NULL, NULL, w);
    double num = 0.0, den = 0.0;
    for (int k = 0; k < ns; k++) {
        double c = rho * u[1 + k] / m->W[k];
        num += (h[k] - 1.0) * w[k];
        den += c * (cp[k] - 1.0);
        f[1 + k] = m->W[k] * w[k] / rho;
    }
    f[0] = -T * num / den;
    free(cp); free(h); free(s); free(w);
}

/* ------------------------------------------------ Jacobian (complex step) */
/* The RHS of or_rhs evaluated in complex arithmetic: every operation in it
 * (polynomials, exp, log, powers, products, the quotient of the T equation)
 * is analytic, so for a real state u and a tiny real step s,
 * Im f(u + i s e_k) / s = df/du_k to rounding, with no subtractive
 * cancellation (the complex-step derivative of Squire and Trapp, 1998).  The
 * NASA-7 range is chosen from the real part of T. */
static void rhs_cplx(const or_mech *m, double rho, const double complex *u, double complex *f) {
    int ns = m->ns;
    double complex T = u[0];
    double complex lnT = clog(T);
    double complex *cp = malloc(sizeof(double complex) * ns);
    double complex *h = malloc(sizeof(double complex) * ns);
    double complex *g = malloc(sizeof(double complex) * ns);
    double complex *c = malloc(sizeof(double complex) * ns);
    double complex *w = malloc(sizeof(double complex) * ns);
    for (int k = 0; k < ns; k++) {
        const double *a = (creal(T) < m->Tmid[k]) ? &m->lo[k * 7] : &m->hi[k * 7];
        cp[k] = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        h[k] = a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
             + a[4] * T * T * T * T / 5.0 + a[5] / T;
        double complex sR = a[0] * lnT + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0
                          + a[4] * T * T * T * T / 4.0 + a[6];
        g[k] = h[k] - sR;
        c[k] = rho * u[1 + k] / m->W[k];
        w[k] = 0.0;
    }
    for (int j = 0; j < m->nr; j++) {
        const or_reaction *r = &m->rx[j];
        double complex kf = r->A * cexp(r->b * lnT) * cexp(-r->Ea / (OR_R_J * T));
        double complex dG = 0.0;
        int dnu = 0;
        for (int i = 0; i < r->n_prod; i++) { dG += r->prod_nu[i] * g[r->prod_sp[i]]; dnu += r->prod_nu[i]; }
        for (int i = 0; i < r->n_reac; i++) { dG -= r->reac_nu[i] * g[r->reac_sp[i]]; dnu -= r->reac_nu[i]; }
        double complex Kc = cexp(-dG) * cexp(dnu * clog(m->pstd / (OR_R_CGS * T)));
        double complex fwd = kf, rev = kf / Kc;
        for (int i = 0; i < r->n_reac; i++)
            for (int n = 0; n < r->reac_nu[i]; n++) fwd *= c[r->reac_sp[i]];
        for (int i = 0; i < r->n_prod; i++)
            for (int n = 0; n < r->prod_nu[i]; n++) rev *= c[r->prod_sp[i]];
        double complex M = 1.0;
        if (r->third_body) {
            M = 0.0;
            for (int k = 0; k < ns; k++) M += r->eff[k] * c[k];
        }
        double complex q = M * (fwd - rev);
        for (int i = 0; i < r->n_reac; i++) w[r->reac_sp[i]] -= r->reac_nu[i] * q;
        for (int i = 0; i < r->n_prod; i++) w[r->prod_sp[i]] += r->prod_nu[i] * q;
    }
    double complex num = 0.0, den = 0.0;
    for (int k = 0; k < ns; k++) {
        num += (h[k] - 1.0) * w[k];
        den += c[k] * (cp[k] - 1.0);
        f[1 + k] = m->W[k] * w[k] / rho;
    }
    f[0] = -T * num / den;
    free(cp); free(h); free(g); free(c); free(w);
}

/* J[i*n + k] = df_i/du_k for u = (T, Y), n = N + 1. */
void or_jacobian(const or_mech *m, double rho, const double *u, double *J) {
    int n = m->ns + 1;
    const double s = 1e-30;
    double complex *uc = malloc(sizeof(double complex) * n);
    double complex *fc = malloc(sizeof(double complex) * n);
    for (int k = 0; k < n; k++) {
        for (int i = 0; i < n; i++) uc[i] = u[i];
        uc[k] += s * I;
        rhs_cplx(m, rho, uc, fc);
        for (int i = 0; i < n; i++) J[i * n + k] = cimag(fc[i]) / s;
    }
    free(uc); free(fc);
}

/* -------------------------------------------------------- LSRK coefficients */
/* Kennedy, Carpenter & Lewis (2000) RK4(3)5[2R+]C: subdiagonal a_{i+1,i},
 * weights b_i and embedded weights bhat_i, as exact rationals. */
static const double LS_A_NUM[4] = {970286171893.0, 6584761158862.0, 2251764453980.0, 26877169314380.0};
static const double LS_A_DEN[4] = {4311952581923.0, 12103376702013.0, 15575788980749.0, 34165994151039.0};
static const double LS_B_NUM[5] = {1153189308089.0, 1772645290293.0, -1672844663538.0, 2114624349019.0, 5198255086312.0};
static const double LS_B_DEN[5] = {22510343858157.0, 4653164025191.0, 4480602732383.0, 3568978502595.0, 14908931495163.0};
static const double LS_BH_NUM[5] = {1016888040809.0, 11231460423587.0, -1563879915014.0, 606302364029.0, 1097981568119.0};
static const double LS_BH_DEN[5] = {7410784769900.0, 58533540763752.0, 6823010717585.0, 971179775848.0, 3980877426909.0};

void or_lsrk_coeffs(double *a, double *b, double *bh) {
    for (int i = 0; i < 4; i++) a[i] = LS_A_NUM[i] / LS_A_DEN[i];
    for (int i = 0; i < 5; i++) { b[i] = LS_B_NUM[i] / LS_B_DEN[i]; bh[i] = LS_BH_NUM[i] / LS_BH_DEN[i]; }
}

/* ----------------------------------------------------------- generic core */
typedef void (*or_rhs_fn)(const void *ctx, const double *u, double *f);

/* One step of Eq. 21 (two registers U, X) plus the error register E:
 *   U <- X + a_{i+1,i} h F_i ;  X <- U + (b_i - a_{i+1,i}) h F_i ;  E += (b_i - bhat_i) h F_i
 * with F_i = f(U), for i = 1..5 (the last stage adds b_5 h F_5 to X). */
static void lsrk_step(or_rhs_fn f, const void *ctx, int n, double h, const double *un,
                      double *unew, double *err_vec, double *U, double *F) {
    double a[4], b[5], bh[5];
    or_lsrk_coeffs(a, b, bh);
    double *X = unew;
    for (int i = 0; i < n; i++) { X[i] = un[i]; U[i] = un[i]; err_vec[i] = 0.0; }
    for (int s = 0; s < 5; s++) {
        f(ctx, U, F);
        for (int i = 0; i < n; i++) err_vec[i] += (b[s] - bh[s]) * h * F[i];
        if (s < 4) {
            for (int i = 0; i < n; i++) {
                U[i] = X[i] + a[s] * h * F[i];
                X[i] = U[i] + (b[s] - a[s]) * h * F[i];
            }
        } else {
            for (int i = 0; i < n; i++) X[i] = X[i] + b[s] * h * F[i];
        }
    }
}

/* The full-storage comparison scheme (the paper's Sec. 4.2.2 compares the
 * low-storage scheme with a Runge-Kutta-Fehlberg integrator): Fehlberg's
 * six-stage 4(5) pair, advancing with the fourth-order weights and
 * estimating the error as the difference to the fifth-order ones.  All
 * stages are kept (k_1..k_6), which is the storage the low-storage scheme
 * avoids.  Coefficients as exact rationals. */
static const double RKF_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
static const double RKF_B4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
static const double RKF_B5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0,
                                 2.0 / 55.0};

void or_rkf45_coeffs(double *a, double *b4, double *b5) {
    for (int i = 0; i < 6; i++) {
        for (int j = 0; j < 5; j++) a[5 * i + j] = RKF_A[i][j];
        b4[i] = RKF_B4[i];
        b5[i] = RKF_B5[i];
    }
}

/* One RKF45 step: k_i = f(u_n + h sum_{j<i} a_ij k_j), unew = u_n + h sum b4_i k_i,
 * err = h sum (b5_i - b4_i) k_i.  K holds the six stage vectors. */
static void rkf45_step(or_rhs_fn f, const void *ctx, int n, double h, const double *un,
                       double *unew, double *err_vec, double *U, double *K) {
    for (int s = 0; s < 6; s++) {
        for (int i = 0; i < n; i++) {
            double acc = 0.0;
            for (int j = 0; j < s; j++) acc += RKF_A[s][j] * K[j * n + i];
            U[i] = un[i] + h * acc;
        }
        f(ctx, U, K + s * n);
    }
    for (int i = 0; i < n; i++) {
        double y4 = 0.0, e = 0.0;
        for (int s = 0; s < 6; s++) {
            y4 += RKF_B4[s] * K[s * n + i];
            e += (RKF_B5[s] - RKF_B4[s]) * K[s * n + i];
        }
        unew[i] = un[i] + h * y4;
        err_vec[i] = h * e;
    }
}

/* The implicit comparator: a Rosenbrock (linearly implicit) step in the
 * Kaps-Rentrop form, with W = I/(gamma h) - J(u_n) and stages
 *   W g1 = f(u_n)
 *   W g2 = f(u_n + a21 g1)              + c21 g1 / h
 *   W g3 = f(u_n + a31 g1 + a32 g2)     + (c31 g1 + c32 g2) / h
 *   W g4 = f(u_n + a31 g1 + a32 g2)     + (c41 g1 + c42 g2 + c43 g3) / h
 * (the fourth stage reuses the third RHS evaluation), u_{n+1} = u_n + sum b_i g_i
 * (fourth order) and the error estimate e = sum e_i g_i (the difference to
 * the embedded third-order solution).  Parameters: Shampine (1982), gamma =
 * 1/2.  For an autonomous RHS the time-derivative terms of the form vanish. */
static const double RO_GAMMA = 0.5;
static const double RO_A21 = 2.0, RO_A31 = 48.0 / 25.0, RO_A32 = 6.0 / 25.0;
static const double RO_C21 = -8.0, RO_C31 = 372.0 / 25.0, RO_C32 = 12.0 / 5.0;
static const double RO_C41 = -112.0 / 125.0, RO_C42 = -54.0 / 125.0, RO_C43 = -2.0 / 5.0;
static const double RO_B[4] = {19.0 / 9.0, 1.0 / 2.0, 25.0 / 108.0, 125.0 / 108.0};
static const double RO_E[4] = {17.0 / 54.0, 7.0 / 36.0, 0.0, 125.0 / 108.0};

typedef void (*or_jac_fn)(const void *ctx, const double *u, double *J);

/* In-place LU factorisation with partial pivoting of the n x n row-major
 * matrix a (P a = L U, whole rows swapped, unit L below the diagonal);
 * piv[k] = row swapped with row k at column k. */
static void lu_factor(int n, double *a, int *piv) {
    for (int k = 0; k < n; k++) {
        int p = k;
        for (int r = k + 1; r < n; r++)
            if (fabs(a[r * n + k]) > fabs(a[p * n + k])) p = r;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; j++) {
                double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t;
            }
        for (int r = k + 1; r < n; r++) {
            double l = a[r * n + k] / a[k * n + k];
            a[r * n + k] = l;
            for (int j = k + 1; j < n; j++) a[r * n + j] -= l * a[k * n + j];
        }
    }
}

/* Solve a x = b in place: b <- P b (the swaps in factorisation order), then
 * L y = P b and U x = y. */
static void lu_solve(int n, const double *a, const int *piv, double *b) {
    for (int k = 0; k < n; k++)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int k = 0; k < n; k++)
        for (int r = k + 1; r < n; r++) b[r] -= a[r * n + k] * b[k];
    for (int k = n - 1; k >= 0; k--) {
        double s = b[k];
        for (int j = k + 1; j < n; j++) s -= a[k * n + j] * b[j];
        b[k] = s / a[k * n + k];
    }
}

static void ros4_step(or_rhs_fn f, or_jac_fn jac, const void *ctx, int n, double h,
                      const double *un, double *unew, double *e) {
    double *W = malloc(sizeof(double) * n * n);
    double *g = malloc(sizeof(double) * n * 4), *y = malloc(sizeof(double) * n);
    double *f3 = malloc(sizeof(double) * n);
    int *piv = calloc((size_t)n, sizeof(int));
    jac(ctx, un, W);
    for (int i = 0; i < n * n; i++) W[i] = -W[i];
    for (int i = 0; i < n; i++) W[i * n + i] += 1.0 / (RO_GAMMA * h);
    lu_factor(n, W, piv);
    double *g1 = g, *g2 = g + n, *g3 = g + 2 * n, *g4 = g + 3 * n;
    f(ctx, un, g1);
    lu_solve(n, W, piv, g1);
    for (int i = 0; i < n; i++) y[i] = un[i] + RO_A21 * g1[i];
    f(ctx, y, g2);
    for (int i = 0; i < n; i++) g2[i] += RO_C21 * g1[i] / h;
    lu_solve(n, W, piv, g2);
    for (int i = 0; i < n; i++) y[i] = un[i] + RO_A31 * g1[i] + RO_A32 * g2[i];
    f(ctx, y, f3);
    for (int i = 0; i < n; i++) g3[i] = f3[i] + (RO_C31 * g1[i] + RO_C32 * g2[i]) / h;
    lu_solve(n, W, piv, g3);
    for (int i = 0; i < n; i++)
        g4[i] = f3[i] + (RO_C41 * g1[i] + RO_C42 * g2[i] + RO_C43 * g3[i]) / h;
    lu_solve(n, W, piv, g4);
    for (int i = 0; i < n; i++) {
        unew[i] = un[i] + RO_B[0] * g1[i] + RO_B[1] * g2[i] + RO_B[2] * g3[i] + RO_B[3] * g4[i];
        e[i] = RO_E[0] * g1[i] + RO_E[1] * g2[i] + RO_E[2] * g3[i] + RO_E[3] * g4[i];
    }
    free(W); free(g); free(y); free(f3); free(piv);
}

/* Eq. 22: WRMS norm of the error with weights from the state at step start. */
static double wrms(int n, const double *e, const double *un, double rtol, double atol) {
    double sum = 0.0;
    for (int i = 0; i < n; i++) {
        double w = e[i] / (rtol * fabs(un[i]) + atol);
        sum += w * w;
    }
    return sqrt(sum / n);
}

/* Eq. 22's step factor with the [1/5, 5] clamp and beta = 0.9; the exponent
 * is 1/(q+1) for an error estimate of order q: 1/4 for the low-storage
 * scheme's third-order estimate, 1/5 for Fehlberg's fourth-order one. */
static double step_factor(double err, double expo) {
    if (err != err) return 0.2;
    if (err == 0.0) return 5.0;
    double fac = 0.9 * pow(err, -expo);
    if ((or_perturb & 2) && expo == 0.25) fac = 0.9 * (1.0 / sqrt(sqrt(err)));
    if (fac < 0.2) fac = 0.2;
    if (fac > 5.0) fac = 5.0;
    return fac;
}

typedef struct { double t, h, err; int accepted; } or_trace;

/* Integrate u over [0, dt]; returns a status code.  h_inout: initial step
 * hint (<= 0 => dt) and, on return, the proposed next step. */
enum { OR_SCHEME_LSRK = 0, OR_SCHEME_RKF45 = 1, OR_SCHEME_ROS4 = 2 };

static void scheme_step(int scheme, or_rhs_fn f, or_jac_fn jac, const void *ctx, int n,
                        double h, const double *un, double *unew, double *e, double *U,
                        double *F) {
    if (scheme == OR_SCHEME_RKF45) rkf45_step(f, ctx, n, h, un, unew, e, U, F);
    else if (scheme == OR_SCHEME_ROS4) ros4_step(f, jac, ctx, n, h, un, unew, e);
    else lsrk_step(f, ctx, n, h, un, unew, e, U, F);
}

static int drive(int scheme, or_rhs_fn f, or_jac_fn jac, const void *ctx, int n, double *u,
                 double dt,
                 double rtol, double atol, int max_steps, int fixed_steps, double *h_inout,
                 int *nacc, int *nrej, or_trace *trace, int trace_cap, int *trace_len) {
    double *unew = malloc(sizeof(double) * n), *e = malloc(sizeof(double) * n);
    double *U = malloc(sizeof(double) * n), *F = malloc(sizeof(double) * n * 6);
    const double expo = scheme == OR_SCHEME_RKF45 ? 0.2 : 0.25;
    int status = OR_OK;
    *nacc = 0; *nrej = 0;
    if (trace_len) *trace_len = 0;
    if (fixed_steps > 0) {
        double h = dt / fixed_steps;
        for (int s = 0; s < fixed_steps; s++) {
            scheme_step(scheme, f, jac, ctx, n, h, u, unew, e, U, F);
            for (int i = 0; i < n; i++) u[i] = unew[i];
            (*nacc)++;
        }
        *h_inout = h;
        free(unew); free(e); free(U); free(F);
        return OR_OK;
    }
    double t = 0.0;
    double h = (*h_inout > 0.0 && *h_inout < dt) ? *h_inout : dt;
    for (;;) {
        int last = 0;
        if (h >= dt - t) { h = dt - t; last = 1; }
        scheme_step(scheme, f, jac, ctx, n, h, u, unew, e, U, F);
        double err = wrms(n, e, u, rtol, atol);
        double fac = step_factor(err, expo);
        int ok = (err <= 1.0);
        if (trace && *trace_len < trace_cap) {
            trace[*trace_len].t = t; trace[*trace_len].h = h;
            trace[*trace_len].err = err; trace[*trace_len].accepted = ok;
            (*trace_len)++;
        }
        if (ok) {
            for (int i = 0; i < n; i++) u[i] = unew[i];
            (*nacc)++;
            if (last) { h = h * fac; break; }
            t = t + h;
        } else {
            (*nrej)++;
        }
        h = h * fac;
        if (*nacc + *nrej >= max_steps) { status = OR_MAXSTEPS; break; }
        if (h < 1e-14 * dt) { status = OR_H_UNDERFLOW; break; }
    }
    *h_inout = h;
    free(unew); free(e); free(U); free(F);
    return status;
}

/* ------------------------------------------------------ chemistry driver */
typedef struct { const or_mech *m; double rho; } chem_ctx;

static void chem_rhs_cb(const void *ctx, const double *u, double *f) {
    const chem_ctx *c = ctx;
    or_rhs(c->m, c->rho, u, f);
}

static void chem_jac_cb(const void *ctx, const double *u, double *J) {
    const chem_ctx *c = ctx;
    or_jacobian(c->m, c->rho, u, J);
}

/* One cell: u (N+1) in/out.  Returns status. */
int or_integrate_cell_scheme(int scheme, const or_mech *m, double rho, double *u, double dt,
                             double rtol, double atol, int max_steps, int fixed_steps,
                             double *h_inout, int *nacc, int *nrej, double *trace_out,
                             int trace_cap, int *trace_len) {
    int n = m->ns + 1;
    for (int i = 0; i < n; i++) if (!isfinite(u[i])) { *nacc = *nrej = 0; return OR_NONFINITE; }
    if (!isfinite(rho)) { *nacc = *nrej = 0; return OR_NONFINITE; }
    chem_ctx ctx = {m, rho};
    or_trace *tr = trace_out ? malloc(sizeof(or_trace) * (trace_cap > 0 ? trace_cap : 1)) : NULL;
    int st = drive(scheme, chem_rhs_cb, chem_jac_cb, &ctx, n, u, dt, rtol, atol, max_steps, fixed_steps,
                   h_inout, nacc, nrej, tr, trace_cap, trace_len);
    if (tr) {
        for (int i = 0; i < *trace_len; i++) {
            trace_out[4 * i + 0] = tr[i].t; trace_out[4 * i + 1] = tr[i].h;
            trace_out[4 * i + 2] = tr[i].err; trace_out[4 * i + 3] = tr[i].accepted;
        }
        free(tr);
    }
    return st;
}

int or_integrate_cell(const or_mech *m, double rho, double *u, double dt, double rtol,
                      double atol, int max_steps, int fixed_steps, double *h_inout,
                      int *nacc, int *nrej, double *trace_out, int trace_cap, int *trace_len) {
    return or_integrate_cell_scheme(OR_SCHEME_LSRK, m, rho, u, dt, rtol, atol, max_steps,
                                    fixed_steps, h_inout, nacc, nrej, trace_out, trace_cap,
                                    trace_len);
}

/* All cells of an SoA state block: state[v*ld + i], rows v = 0 T, 1..N Y_k,
 * N+1 rho (read only), N+2 h (in: step hint, <= 0 => dt; out: next step).
 * counts (may be NULL) receives n_acc in [i] and n_rej in [n + i]. */
int or_integrate_scheme(int scheme, const or_mech *m, double *state, int64_t ld, int64_t n,
                        double dt, double rtol, double atol, int max_steps, int fixed_steps,
                        int nthreads, int32_t *status, int32_t *counts) {
    int N = m->ns;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t i = 0; i < n; i++) {
        double u[1 + 64];
        for (int v = 0; v <= N; v++) u[v] = state[v * ld + i];
        double rho = state[(N + 1) * ld + i];
        double h = state[(N + 2) * ld + i];
        int na = 0, nr = 0;
        int st = or_integrate_cell_scheme(scheme, m, rho, u, dt, rtol, atol, max_steps,
                                          fixed_steps, &h, &na, &nr, NULL, 0, NULL);
        if (st != OR_NONFINITE) {
            for (int v = 0; v <= N; v++) state[v * ld + i] = u[v];
            state[(N + 2) * ld + i] = h;
        }
        if (status) status[i] = st;
        if (counts) { counts[i] = na; counts[n + i] = nr; }
    }
    return 0;
}

int or_integrate(const or_mech *m, double *state, int64_t ld, int64_t n, double dt,
                 double rtol, double atol, int max_steps, int fixed_steps, int nthreads,
                 int32_t *status, int32_t *counts) {
    return or_integrate_scheme(OR_SCHEME_LSRK, m, state, ld, n, dt, rtol, atol, max_steps,
                               fixed_steps, nthreads, status, counts);
}

/* ------------------------------------- coupling to the flow (Sec. 2.2.1) */
/* Mixture internal energy e = sum_k Y_k (h_k - R T / W_k) [erg/g] and
 * c_v = sum_k Y_k (cp_k - R / W_k) [erg/(g K)] from the NASA-7 fits. */
void or_energy(const or_mech *m, double T, const double *Y, double *e, double *cv) {
    int N = m->ns;
    double cp[64], h[64], sR[64];
    or_thermo(m, T, cp, h, sR);
    double se = 0.0, sc = 0.0;
    for (int k = 0; k < N; k++) {
        se += Y[k] * (h[k] - 1.0) / m->W[k];
        sc += Y[k] * (cp[k] - 1.0) / m->W[k];
    }
    *e = OR_R_CGS * T * se;
    *cv = OR_R_CGS * sc;
}

/* Temperature from conserved quantities: Newton iteration on
 * e(T, Y) = e_target from T0 (<= 0: 1000 K), T <- T - (e(T) - e_target)/c_v(T),
 * until |dT| <= 1e-12 T; returns the iterations taken, or -1 if 50 were not
 * enough or T left (0, inf). */
int or_calculate_T(const or_mech *m, const double *Y, double e_target, double T0, double *T) {
    double t = T0 > 0.0 ? T0 : 1000.0;
    for (int it = 1; it <= 50; it++) {
        double e, cv;
        or_energy(m, t, Y, &e, &cv);
        double dT = (e - e_target) / cv;
        t -= dT;
        if (!(t > 0.0) || !isfinite(t)) return -1;
        if (fabs(dT) <= 1e-12 * t) { *T = t; return it; }
    }
    *T = t;
    return -1;
}

/* One reaction step of the split scheme on conserved variables (SoA rows:
 * rho, rho u, rho v, rho w, rho E, rho Y_1..rho Y_N, T, h): T from
 * e = E - |u|^2/2 by Newton (the T row is the initial guess), the chemistry
 * ODE over dt at constant rho and e, then rho Y_k and the T and h rows
 * written back; rho, momentum and rho E are unchanged.  Status 4 marks a
 * cell whose Newton iteration failed (left unchanged). */
int or_react_conserved(const or_mech *m, double *cons, int64_t ld, int64_t n, double dt,
                       double rtol, double atol, int nthreads, int32_t *status, int32_t *counts) {
    int N = m->ns;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t i = 0; i < n; i++) {
        double rho = cons[i];
        double mu = cons[1 * ld + i], mv = cons[2 * ld + i], mw = cons[3 * ld + i];
        double E = cons[4 * ld + i] / rho;
        double e = E - 0.5 * (mu * mu + mv * mv + mw * mw) / (rho * rho);
        double u[1 + 64];
        for (int k = 0; k < N; k++) u[1 + k] = cons[(5 + k) * ld + i] / rho;
        double T;
        int it = or_calculate_T(m, u + 1, e, cons[(5 + N) * ld + i], &T);
        int na = 0, nr = 0, st;
        if (it < 0) {
            st = 4;
        } else {
            u[0] = T;
            double h = cons[(6 + N) * ld + i];
            st = or_integrate_cell(m, rho, u, dt, rtol, atol, 100000, 0, &h, &na, &nr, NULL, 0,
                                   NULL);
            if (st != OR_NONFINITE) {
                for (int k = 0; k < N; k++) cons[(5 + k) * ld + i] = rho * u[1 + k];
                cons[(5 + N) * ld + i] = u[0];
                cons[(6 + N) * ld + i] = h;
            }
        }
        if (status) status[i] = st;
        if (counts) { counts[i] = na; counts[n + i] = nr; }
    }
    return 0;
}

/* ---------------------------------------------- linear test problems */
typedef struct { int n; const double *A; } lin_ctx;

static void lin_rhs_cb(const void *ctx, const double *u, double *f) {
    const lin_ctx *c = ctx;
    for (int i = 0; i < c->n; i++) {
        double s = 0.0;
        for (int j = 0; j < c->n; j++) s += c->A[i * c->n + j] * u[j];
        f[i] = s;
    }
}

static void lin_jac_cb(const void *ctx, const double *u, double *J) {
    const lin_ctx *c = ctx;
    (void)u;
    for (int i = 0; i < c->n * c->n; i++) J[i] = c->A[i];
}

/* u' = A u with the same step, controller and driver as the chemistry path. */
int or_integrate_linear_scheme(int scheme, int n, const double *A, double *u, double dt,
                               double rtol, double atol, int max_steps, int fixed_steps,
                               double *h_inout, int *nacc, int *nrej, double *trace_out,
                               int trace_cap, int *trace_len) {
    lin_ctx ctx = {n, A};
    or_trace *tr = trace_out ? malloc(sizeof(or_trace) * (trace_cap > 0 ? trace_cap : 1)) : NULL;
    int st = drive(scheme, lin_rhs_cb, lin_jac_cb, &ctx, n, u, dt, rtol, atol, max_steps, fixed_steps,
                   h_inout, nacc, nrej, tr, trace_cap, trace_len);
    if (tr) {
        for (int i = 0; i < *trace_len; i++) {
            trace_out[4 * i + 0] = tr[i].t; trace_out[4 * i + 1] = tr[i].h;
            trace_out[4 * i + 2] = tr[i].err; trace_out[4 * i + 3] = tr[i].accepted;
        }
        free(tr);
    }
    return st;
}

int or_integrate_linear(int n, const double *A, double *u, double dt, double rtol, double atol,
                        int max_steps, int fixed_steps, double *h_inout, int *nacc, int *nrej,
                        double *trace_out, int trace_cap, int *trace_len) {
    return or_integrate_linear_scheme(OR_SCHEME_LSRK, n, A, u, dt, rtol, atol, max_steps,
                                      fixed_steps, h_inout, nacc, nrej, trace_out, trace_cap,
                                      trace_len);
}
