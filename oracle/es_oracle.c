/*
 * es_oracle.c -- plain CPU FP64 oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Li, Duan & Tang, "High-order accurate entropy stable adaptive moving mesh
 * finite difference schemes for (multi-component) compressible Euler equations
 * with the stiffened equation of state", arXiv 2202.07989.
 *
 * Every routine follows the cited passage in the paper's order and notation,
 * without blocking, fusion or reordering.  Where the paper is silent the
 * readings listed in the design notes are used (they are named here as
 * "reading: ..." next to the code they affect).  Nothing here is tuned.
 */
#include "es_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXC 6          /* nc <= N + d + 1 = 6 */

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONPHYS = -4, ORC_ETANGLE = -5 };

/* ------------------------------------------------------------------------ */
/* grid helpers                                                             */
/* ------------------------------------------------------------------------ */
static int npad(const orc_grid *g, int k) { return k < g->dim ? g->n[k] + 2 * g->ng : 1; }
static int lo_(const orc_grid *g, int k) { return k < g->dim ? g->ng : 0; }
static int hi_(const orc_grid *g, int k) { return lo_(g, k) + (k < g->dim ? g->n[k] : 1); }
long orc_npoints(const orc_grid *g) { return (long)npad(g, 0) * npad(g, 1) * npad(g, 2); }
static long at(const orc_grid *g, int i0, int i1, int i2)
{
    return ((long)i2 * npad(g, 1) + i1) * npad(g, 0) + i0;
}
static long stride_(const orc_grid *g, int k)
{
    return k == 0 ? 1 : (k == 1 ? (long)npad(g, 0) : (long)npad(g, 0) * npad(g, 1));
}
int orc_ncomp(const orc_grid *g) { return g->nspec + g->dim + 1; }
static double gas_const(const orc_grid *g, int l) { return g->cv[l] * (g->gamma[l] - 1.0); }
static double cell_volume(const orc_grid *g)
{
    double dv = 1.0;
    for (int k = 0; k < g->dim; k++) dv *= g->dxi[k];
    return dv;
}
static int valid_grid(const orc_grid *g)
{
    if (!g || (g->dim != 2 && g->dim != 3) || (g->nspec != 1 && g->nspec != 2)) return 0;
    if (g->ng < 3 || g->w < 1 || g->w > 3) return 0;
    for (int k = 0; k < g->dim; k++) {
        if (g->n[k] < 1 || !(g->dxi[k] > 0)) return 0;
        for (int s = 0; s < 2; s++)
            if (g->bc[k][s] < 0 || g->bc[k][s] > 3) return 0;
        /* a direction is periodic on both faces or on neither */
        if ((g->bc[k][0] == 0) != (g->bc[k][1] == 0)) return 0;
        if (g->bc[k][0] != 0 && !(g->wall[k][1] > g->wall[k][0])) return 0;
    }
    if (g->dim == 2 && g->n[2] != 1) return 0;
    if (!(g->sign_tol >= 0.0 && g->sign_tol < 1.0)) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2, constants alpha_{w,m} of the 2w-th order EC flux: they solve */
/* sum_m m alpha = 1 and sum_m m^(2s-1) alpha = 0, s = 2..w (LeFloch et al.) */
/* ------------------------------------------------------------------------ */
void orc_alpha(int w, double alpha[3])
{
    alpha[0] = alpha[1] = alpha[2] = 0.0;
    if (w == 1) { alpha[0] = 1.0; }
    else if (w == 2) { alpha[0] = 4.0 / 3.0; alpha[1] = -1.0 / 6.0; }
    else if (w == 3) { alpha[0] = 3.0 / 2.0; alpha[1] = -3.0 / 10.0; alpha[2] = 1.0 / 30.0; }
}

/* ------------------------------------------------------------------------ */
/* Section 3.3.1, logarithmic mean {a}^ln = [[a]] / [[ln a]].               */
/* Reading (paper silent on evaluation): with zeta = al/ar,                 */
/* f = (zeta-1)/(zeta+1), u = f^2, the ratio ln(zeta)/(2f) is replaced by    */
/* its series 1 + u/3 + u^2/5 + u^3/7 when u < 1e-4; {a}^ln = (al+ar)/(2F).  */
/* ------------------------------------------------------------------------ */
double orc_logmean(double al, double ar)
{
    if (al == ar) return al;
    double zeta = al / ar;
    double f = (zeta - 1.0) / (zeta + 1.0);
    double u = f * f;
    double F;
    if (u < 1.0e-4) F = 1.0 + u / 3.0 + u * u / 5.0 + u * u * u / 7.0;
    else F = log(zeta) / (2.0 * f);
    return (al + ar) / (2.0 * F);
}

/* ------------------------------------------------------------------------ */
/* Section 1, system and stiffened EOS: U = (rho_1..rho_N, rho v, E),        */
/* rho e = sum_l (c_vl rho_l T + p_inf,l), p = sum_l (rho_l R_l T - p_inf,l),*/
/* R_l = c_vl (Gamma_l - 1).                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    double rho[2], rhot, v[3], T, p;
} prim_t;

static int prim_of(const orc_grid *g, const double *U, prim_t *q)
{
    int N = g->nspec, d = g->dim;
    double rhot = 0.0, cvrho = 0.0, pinf = 0.0, kin = 0.0;
    int ok = 1;
    memset(q, 0, sizeof(*q));
    for (int l = 0; l < N; l++) {
        q->rho[l] = U[l];
        rhot += U[l];
        cvrho += g->cv[l] * U[l];
        pinf += g->pinf[l];
        if (!(U[l] > 0.0)) ok = 0;
    }
    q->rhot = rhot;
    for (int m = 0; m < d; m++) {
        q->v[m] = U[N + m] / rhot;
        kin += 0.5 * U[N + m] * q->v[m];
    }
    double rhoe = U[N + d] - kin;
    q->T = (rhoe - pinf) / cvrho;
    q->p = 0.0;
    for (int l = 0; l < N; l++) q->p += q->rho[l] * gas_const(g, l) * q->T - g->pinf[l];
    if (!(q->T > 0.0) || !isfinite(q->T) || !isfinite(q->p)) ok = 0;
    for (int m = 0; m < d; m++) if (!isfinite(q->v[m])) ok = 0;
    return ok ? ORC_OK : ORC_ENONPHYS;
}

int orc_prim(const orc_grid *g, const double *U, double *rho, double *v, double *T, double *p)
{
    prim_t q;
    int rc = prim_of(g, U, &q);
    for (int l = 0; l < g->nspec; l++) rho[l] = q.rho[l];
    for (int m = 0; m < g->dim; m++) v[m] = q.v[m];
    *T = q.T;
    *p = q.p;
    return rc;
}

/* mixture Gamma = sum Gamma_l c_vl rho_l / sum c_vl rho_l (Section 1) and   */
/* mixture gas constant R = sum (Gamma_l - 1) c_vl rho_l / rho (Section 3.4) */
static double mix_gamma(const orc_grid *g, const prim_t *q)
{
    double a = 0.0, b = 0.0;
    for (int l = 0; l < g->nspec; l++) {
        a += g->gamma[l] * g->cv[l] * q->rho[l];
        b += g->cv[l] * q->rho[l];
    }
    return a / b;
}
static double mix_R(const orc_grid *g, const prim_t *q)
{
    double a = 0.0;
    for (int l = 0; l < g->nspec; l++) a += gas_const(g, l) * q->rho[l];
    return a / q->rhot;
}

/* sound speed c^2 = R Gamma T (Section 3.4) */
double orc_sound_speed(const orc_grid *g, const double *U)
{
    prim_t q;
    prim_of(g, U, &q);
    return sqrt(mix_R(g, &q) * mix_gamma(g, &q) * q.T);
}

/* Sections 3.3.1 / 3.3.2: entropy variables                                */
/* V = (-S_l - |v|^2/(2T) + c_vl Gamma_l, v/T, -1/T),                        */
/* S_l = c_vl ln T - R_l ln rho_l.                                          */
static void entropy_vars_of(const orc_grid *g, const prim_t *q, double *V)
{
    int N = g->nspec, d = g->dim;
    double v2 = 0.0;
    for (int m = 0; m < d; m++) v2 += q->v[m] * q->v[m];
    for (int l = 0; l < N; l++) {
        double S = g->cv[l] * log(q->T) - gas_const(g, l) * log(q->rho[l]);
        V[l] = -S - v2 / (2.0 * q->T) + g->cv[l] * g->gamma[l];
    }
    for (int m = 0; m < d; m++) V[N + m] = q->v[m] / q->T;
    V[N + d] = -1.0 / q->T;
}

int orc_entropy_vars(const orc_grid *g, const double *U, double *V)
{
    prim_t q;
    int rc = prim_of(g, U, &q);
    entropy_vars_of(g, &q, V);
    return rc;
}

/* eta = -sum_l rho_l S_l (EQ entropypair) */
static double entropy_of(const orc_grid *g, const prim_t *q)
{
    double e = 0.0;
    for (int l = 0; l < g->nspec; l++) {
        double S = g->cv[l] * log(q->T) - gas_const(g, l) * log(q->rho[l]);
        e -= q->rho[l] * S;
    }
    return e;
}
double orc_entropy(const orc_grid *g, const double *U)
{
    prim_t q;
    prim_of(g, U, &q);
    return entropy_of(g, &q);
}

/* phi = sum_l (R_l rho_l - p_inf,l / T) (eq potentialN1 / potentialN2) */
static double potential_of(const orc_grid *g, const prim_t *q)
{
    double phi = 0.0;
    for (int l = 0; l < g->nspec; l++) phi += gas_const(g, l) * q->rho[l] - g->pinf[l] / q->T;
    return phi;
}
double orc_potential(const orc_grid *g, const double *U)
{
    prim_t q;
    prim_of(g, U, &q);
    return potential_of(g, &q);
}

/* physical flux F_j (eq ConserLaw) */
void orc_phys_flux(const orc_grid *g, const double *U, int j, double *F)
{
    int N = g->nspec, d = g->dim;
    prim_t q;
    prim_of(g, U, &q);
    for (int l = 0; l < N; l++) F[l] = q.rho[l] * q.v[j];
    for (int m = 0; m < d; m++) F[N + m] = q.rhot * q.v[j] * q.v[m] + (m == j ? q.p : 0.0);
    F[N + d] = (U[N + d] + q.p) * q.v[j];
}

/* ------------------------------------------------------------------------ */
/* Section 3.3, two-point EC flux (eq ECfluxMM):                             */
/*   F = 1/2 (n_t,l + n_t,r) Utilde + sum_j 1/2 (n_j,l + n_j,r) Ftilde_j,    */
/* with Utilde and Ftilde_1 the closed forms of Sections 3.3.1/3.3.2 in the  */
/* parameter vector z = (rho_1..rho_N, v, 1/T); Ftilde_j, j > 1, are the     */
/* same with the roles of v_1 and v_j exchanged.                            */
/* ------------------------------------------------------------------------ */
static void ec_flux_of(const orc_grid *g, const prim_t *l, const prim_t *r,
                       const double *ml, const double *mr, double *F)
{
    int N = g->nspec, d = g->dim, nc = N + d + 1;
    double rln[2], rmean[2], vmean[3], v2mean[3];
    double bl = 1.0 / l->T, br = 1.0 / r->T;
    double bmean = 0.5 * (bl + br);
    double bln = orc_logmean(bl, br);
    double pinf = 0.0, sum_rln = 0.0, sum_v2 = 0.0, sum_vsq = 0.0;
    for (int s = 0; s < N; s++) {
        rln[s] = orc_logmean(l->rho[s], r->rho[s]);
        rmean[s] = 0.5 * (l->rho[s] + r->rho[s]);
        sum_rln += rln[s];
        pinf += g->pinf[s];
    }
    for (int m = 0; m < d; m++) {
        vmean[m] = 0.5 * (l->v[m] + r->v[m]);
        v2mean[m] = 0.5 * (l->v[m] * l->v[m] + r->v[m] * r->v[m]);  /* {v_m^2} */
        sum_v2 += v2mean[m];
        sum_vsq += vmean[m] * vmean[m];                              /* {v_m}^2 */
    }
    double Ut[MAXC], Ft[3][MAXC];
    /* Utilde */
    for (int s = 0; s < N; s++) Ut[s] = rln[s];
    for (int m = 0; m < d; m++) Ut[N + m] = vmean[m] * sum_rln;
    Ut[N + d] = 0.0;
    for (int s = 0; s < N; s++) Ut[N + d] += rln[s] * (g->cv[s] / bln - 0.5 * sum_v2);
    Ut[N + d] += sum_rln * sum_vsq + pinf;
    /* Ftilde_j */
    double Rrho = 0.0;
    for (int s = 0; s < N; s++) Rrho += gas_const(g, s) * rmean[s];
    for (int j = 0; j < d; j++) {
        double sumF = 0.0;
        for (int s = 0; s < N; s++) { Ft[j][s] = rln[s] * vmean[j]; sumF += Ft[j][s]; }
        for (int m = 0; m < d; m++) {
            Ft[j][N + m] = vmean[m] * sumF;
            if (m == j) Ft[j][N + m] += Rrho / bmean - pinf;
        }
        Ft[j][N + d] = 0.0;
        for (int s = 0; s < N; s++) Ft[j][N + d] += Ft[j][s] * (g->cv[s] / bln - 0.5 * sum_v2);
        for (int m = 0; m < d; m++) Ft[j][N + d] += vmean[m] * Ft[j][N + m];
        Ft[j][N + d] += pinf * vmean[j];
    }
    for (int c = 0; c < nc; c++) {
        F[c] = 0.5 * (ml[0] + mr[0]) * Ut[c];
        for (int j = 0; j < d; j++) F[c] += 0.5 * (ml[1 + j] + mr[1 + j]) * Ft[j][c];
    }
}

/* Sum of the absolute values of the summands of each component of the pair
   flux of ec_flux_of (same printed form n_t Utilde + sum_j n_j Ftilde_j):
   the size of the terms whose rounding a lower-precision evaluation of the
   flux suffers (test infrastructure for the mixed-precision bound). */
static void ec_flux_mag_of(const orc_grid *g, const prim_t *l, const prim_t *r,
                           const double *ml, const double *mr, double *Fm)
{
    int N = g->nspec, d = g->dim, nc = N + d + 1;
    double rln[2], rmean[2], vmean[3];
    double bl = 1.0 / l->T, br = 1.0 / r->T;
    double bmean = 0.5 * (bl + br);
    double bln = orc_logmean(bl, br);
    double pinf = 0.0, sum_rln = 0.0, sum_v2 = 0.0, sum_vsq = 0.0;
    for (int s = 0; s < N; s++) {
        rln[s] = orc_logmean(l->rho[s], r->rho[s]);
        rmean[s] = 0.5 * (l->rho[s] + r->rho[s]);
        sum_rln += rln[s];
        pinf += g->pinf[s];
    }
    for (int m = 0; m < d; m++) {
        vmean[m] = 0.5 * (l->v[m] + r->v[m]);
        sum_v2 += 0.5 * (l->v[m] * l->v[m] + r->v[m] * r->v[m]);
        sum_vsq += vmean[m] * vmean[m];
    }
    double Ut[MAXC], Ft[3][MAXC];
    for (int s = 0; s < N; s++) Ut[s] = rln[s];
    for (int m = 0; m < d; m++) Ut[N + m] = fabs(vmean[m]) * sum_rln;
    Ut[N + d] = 0.0;
    for (int s = 0; s < N; s++) Ut[N + d] += rln[s] * (g->cv[s] / bln + 0.5 * sum_v2);
    Ut[N + d] += sum_rln * sum_vsq + pinf;
    double Rrho = 0.0;
    for (int s = 0; s < N; s++) Rrho += gas_const(g, s) * rmean[s];
    for (int j = 0; j < d; j++) {
        double sumF = 0.0;
        for (int s = 0; s < N; s++) { Ft[j][s] = rln[s] * fabs(vmean[j]); sumF += Ft[j][s]; }
        for (int m = 0; m < d; m++) {
            Ft[j][N + m] = fabs(vmean[m]) * sumF;
            if (m == j) Ft[j][N + m] += Rrho / bmean + pinf;
        }
        Ft[j][N + d] = 0.0;
        for (int s = 0; s < N; s++) Ft[j][N + d] += Ft[j][s] * (g->cv[s] / bln + 0.5 * sum_v2);
        for (int m = 0; m < d; m++) Ft[j][N + d] += fabs(vmean[m]) * Ft[j][N + m];
        Ft[j][N + d] += pinf * fabs(vmean[j]);
    }
    for (int c = 0; c < nc; c++) {
        Fm[c] = fabs(0.5 * (ml[0] + mr[0])) * Ut[c];
        for (int j = 0; j < d; j++) Fm[c] += fabs(0.5 * (ml[1 + j] + mr[1 + j])) * Ft[j][c];
    }
}

int orc_ec_flux(const orc_grid *g, const double *Ul, const double *Ur,
                const double *ml, const double *mr, double *F)
{
    prim_t l, r;
    int a = prim_of(g, Ul, &l), b = prim_of(g, Ur, &r);
    ec_flux_of(g, &l, &r, ml, mr, F);
    return a ? a : b;
}

/* ------------------------------------------------------------------------ */
/* Section 3.4, rotation matrix T (eq rotamatrix).  Reading: the first row   */
/* of the velocity block is n/|n| (atan2 semantics for theta and phi), and   */
/* theta = 0 when n_1 = n_2 = 0.  In 2D the block is [[c, s], [-s, c]].      */
/* ------------------------------------------------------------------------ */
static void rot_block(int d, const double *n, double Tv[3][3])
{
    double nn = 0.0;
    for (int j = 0; j < d; j++) nn += n[j] * n[j];
    nn = sqrt(nn);
    memset(Tv, 0, 9 * sizeof(double));
    if (!(nn > 0.0)) { for (int j = 0; j < 3; j++) Tv[j][j] = 1.0; return; }
    if (d == 2) {
        double c = n[0] / nn, s = n[1] / nn;
        Tv[0][0] = c;  Tv[0][1] = s;
        Tv[1][0] = -s; Tv[1][1] = c;
        return;
    }
    double r12 = sqrt(n[0] * n[0] + n[1] * n[1]);
    double ct = 1.0, st = 0.0;
    if (r12 > 0.0) { ct = n[0] / r12; st = n[1] / r12; }
    double sp = n[2] / nn, cp = r12 / nn;
    Tv[0][0] = cp * ct;  Tv[0][1] = cp * st;  Tv[0][2] = sp;
    Tv[1][0] = -st;      Tv[1][1] = ct;       Tv[1][2] = 0.0;
    Tv[2][0] = -sp * ct; Tv[2][1] = -sp * st; Tv[2][2] = cp;
}

void orc_rotation(const orc_grid *g, const double *n, double *T)
{
    int N = g->nspec, d = g->dim, nc = N + d + 1;
    double Tv[3][3];
    rot_block(d, n, Tv);
    memset(T, 0, (size_t)nc * nc * sizeof(double));
    for (int s = 0; s < N; s++) T[s * nc + s] = 1.0;
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) T[(N + a) * nc + N + b] = Tv[a][b];
    T[(N + d) * nc + N + d] = 1.0;
}

/* ------------------------------------------------------------------------ */
/* Section 3.4, scaled right eigenvectors R at the interface, built from the */
/* paper's averaged values, evaluated at the rotated state (velocity T v).   */
/* N = 1: R = Rtilde diag(rho/(2 Gamma R), rho/(c_v Gamma), rho T, rho T,    */
/*        rho/(2 Gamma R))^(1/2), averages rho = {rho}^ln, v = {v},          */
/*        p + p_inf = {rho}^ln / {rho/(p + p_inf)}^ln.                      */
/* N = 2: R = Rtilde D, D = sqrt(rho/(Gamma R)) diag(1/sqrt2, D^Y, 1, 1,     */
/*        1/sqrt2), averages rho_l = {rho_l}^ln, rho = {rho}^ln, v = {v},    */
/*        T = 1/{1/T}^ln, R = {R}, Gamma = {Gamma},                          */
/*        sum rho_l h_l = sum (c_vl rho_l T + p_inf,l) + {p}.                */
/* Reading: Y_l = rho_l / rho with the averaged values, and                  */
/*        d_l = (c_vl + R_l - Gamma c_vl) T.                                */
/* In 2D the v_3 row and the second tangential column are dropped.           */
/* s = |n_t + v.n| + |n| c is max_m |n_t + L_k lambda_m| (eq HOstable).      */
/* ------------------------------------------------------------------------ */
static void frame_of(const orc_grid *g, const prim_t *ql, const prim_t *qr,
                     const double *m, double *Rm, double *s_out, double Tv[3][3])
{
    int N = g->nspec, d = g->dim, nc = N + d + 1;
    double n[3] = {0, 0, 0}, nn = 0.0;
    for (int j = 0; j < d; j++) { n[j] = m[1 + j]; nn += n[j] * n[j]; }
    nn = sqrt(nn);
    rot_block(d, n, Tv);

    double vbar[3] = {0, 0, 0}, vhat[3] = {0, 0, 0};
    for (int j = 0; j < d; j++) vbar[j] = 0.5 * (ql->v[j] + qr->v[j]);
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) vhat[a] += Tv[a][b] * vbar[b];
    double vv = 0.0;
    for (int j = 0; j < d; j++) vv += vhat[j] * vhat[j];

    double Rt[MAXC][MAXC];   /* Rtilde, row = component, column = wave */
    double cbar, Rscaled[MAXC][MAXC];
    memset(Rt, 0, sizeof(Rt));
    memset(Rscaled, 0, sizeof(Rscaled));

    if (N == 1) {
        double G = g->gamma[0], cv = g->cv[0], Rg = gas_const(g, 0), pinf = g->pinf[0];
        double rho = orc_logmean(ql->rho[0], qr->rho[0]);
        double ppinf = rho / orc_logmean(ql->rho[0] / (ql->p + pinf), qr->rho[0] / (qr->p + pinf));
        double T = ppinf / (Rg * rho);
        double c = sqrt(G * ppinf / rho);
        double H = G * cv * T + 0.5 * vv;   /* (E + p)/rho of the averaged state */
        cbar = c;
        /* columns: lambda = vhat1 - c, vhat1 (entropy), tangential(s), vhat1 + c */
        int cm = 0, ce = 1, cp = nc - 1;     /* column of the + wave */
        Rt[0][cm] = 1.0; Rt[0][ce] = 1.0; Rt[0][cp] = 1.0;
        for (int j = 0; j < d; j++) {
            Rt[1 + j][cm] = vhat[j] - (j == 0 ? c : 0.0);
            Rt[1 + j][ce] = vhat[j];
            Rt[1 + j][cp] = vhat[j] + (j == 0 ? c : 0.0);
        }
        Rt[1 + d][cm] = H - c * vhat[0];
        Rt[1 + d][ce] = 0.5 * vv;
        Rt[1 + d][cp] = H + c * vhat[0];
        for (int t = 1; t < d; t++) {        /* tangential columns 2..d */
            Rt[1 + t][1 + t] = 1.0;
            Rt[1 + d][1 + t] = vhat[t];
        }
        double sc[MAXC];
        sc[cm] = sqrt(rho / (2.0 * G * Rg));
        sc[ce] = sqrt(rho / (cv * G));
        for (int t = 1; t < d; t++) sc[1 + t] = sqrt(rho * T);
        sc[cp] = sqrt(rho / (2.0 * G * Rg));
        for (int a = 0; a < nc; a++)
            for (int b = 0; b < nc; b++) Rscaled[a][b] = Rt[a][b] * sc[b];
    } else {
        double rl[2], Rl[2], cvl[2];
        for (int s = 0; s < 2; s++) {
            rl[s] = orc_logmean(ql->rho[s], qr->rho[s]);
            Rl[s] = gas_const(g, s);
            cvl[s] = g->cv[s];
        }
        double rho = orc_logmean(ql->rhot, qr->rhot);
        double T = 1.0 / orc_logmean(1.0 / ql->T, 1.0 / qr->T);
        double Rm = 0.5 * (mix_R(g, ql) + mix_R(g, qr));
        double G = 0.5 * (mix_gamma(g, ql) + mix_gamma(g, qr));
        double rhoh = 0.5 * (ql->p + qr->p);
        for (int s = 0; s < 2; s++) rhoh += cvl[s] * rl[s] * T + g->pinf[s];
        double H = rhoh / rho + 0.5 * vv;
        double Y[2] = {rl[0] / rho, rl[1] / rho};
        double dl[2];
        for (int s = 0; s < 2; s++) dl[s] = (cvl[s] + Rl[s] - G * cvl[s]) * T;
        double c = sqrt(G * Rm * T);
        cbar = c;
        /* columns: 0 (v1 - c), 1, 2 (species), 3..d+1 (tangential), d+2 (v1 + c) */
        int cp = nc - 1;
        Rt[0][0] = Y[0]; Rt[1][0] = Y[1];
        Rt[0][1] = 1.0;  Rt[1][2] = 1.0;
        Rt[0][cp] = Y[0]; Rt[1][cp] = Y[1];
        for (int j = 0; j < d; j++) {
            Rt[2 + j][0] = vhat[j] - (j == 0 ? c : 0.0);
            Rt[2 + j][1] = vhat[j];
            Rt[2 + j][2] = vhat[j];
            Rt[2 + j][cp] = vhat[j] + (j == 0 ? c : 0.0);
        }
        Rt[2 + d][0] = H - c * vhat[0];
        Rt[2 + d][1] = 0.5 * vv - dl[0] / (G - 1.0);
        Rt[2 + d][2] = 0.5 * vv - dl[1] / (G - 1.0);
        Rt[2 + d][cp] = H + c * vhat[0];
        for (int t = 1; t < d; t++) {
            Rt[2 + t][2 + t] = c;
            Rt[2 + d][2 + t] = c * vhat[t];
        }
        double Dm[MAXC][MAXC];
        memset(Dm, 0, sizeof(Dm));
        double sq = sqrt(rho / (G * Rm));
        double yy = sqrt(Y[0] * Y[1]);
        Dm[0][0] = sq / sqrt(2.0);
        Dm[1][1] = -sq * yy * sqrt(G * Rl[1] / Rl[0]);
        Dm[1][2] = sq * Y[0] * sqrt(G - 1.0);
        Dm[2][1] = sq * yy * sqrt(G * Rl[0] / Rl[1]);
        Dm[2][2] = sq * Y[1] * sqrt(G - 1.0);
        for (int t = 1; t < d; t++) Dm[2 + t][2 + t] = sq;
        Dm[cp][cp] = sq / sqrt(2.0);
        for (int a = 0; a < nc; a++)
            for (int b = 0; b < nc; b++) {
                double acc = 0.0;
                for (int e = 0; e < nc; e++) acc += Rt[a][e] * Dm[e][b];
                Rscaled[a][b] = acc;
            }
    }
    for (int a = 0; a < nc; a++)
        for (int b = 0; b < nc; b++) Rm[a * nc + b] = Rscaled[a][b];
    double vn = 0.0;
    for (int j = 0; j < d; j++) vn += vbar[j] * n[j];
    *s_out = fabs(m[0] + vn) + nn * cbar;
}

int orc_interface_frame(const orc_grid *g, const double *Ul, const double *Ur,
                        const double *m, double *R, double *s)
{
    prim_t l, r;
    double Tv[3][3];
    int a = prim_of(g, Ul, &l), b = prim_of(g, Ur, &r);
    frame_of(g, &l, &r, m, R, s, Tv);
    return a ? a : b;
}

/* ------------------------------------------------------------------------ */
/* Appendix A, fifth-order multi-resolution WENO.  q[0..4] = W_{j-2..j+2};  */
/* returns W^WENO_{j+1/2}.  h_m are the Legendre expansions evaluated at     */
/* (xi - xi_j)/dxi = 1/2; beta_2, beta_3 are the printed closed forms.      */
/* ------------------------------------------------------------------------ */
double orc_mr5(const double *q, const double *chi, double eps)
{
    double Wm2 = q[0], Wm1 = q[1], W0 = q[2], Wp1 = q[3], Wp2 = q[4];
    double a1 = W0;
    double a2 = (Wp1 - Wm1) / 2.0;
    double a3 = (Wm1 - 2.0 * W0 + Wp1) / 2.0;
    double b1 = W0;
    double b2 = (11.0 * Wm2 - 82.0 * Wm1 + 82.0 * Wp1 - 11.0 * Wp2) / 120.0;
    double b3 = (-3.0 * Wm2 + 40.0 * Wm1 - 74.0 * W0 + 40.0 * Wp1 - 3.0 * Wp2) / 56.0;
    double b4 = (-Wm2 + 2.0 * Wm1 - 2.0 * Wp1 + Wp2) / 12.0;
    double b5 = (Wm2 - 4.0 * Wm1 + 6.0 * W0 - 4.0 * Wp1 + Wp2) / 24.0;

    double d1 = (W0 - Wm1) * (W0 - Wm1), d2 = (Wp1 - W0) * (Wp1 - W0);
    double beta1 = d1 < d2 ? d1 : d2;
    double beta2 = a2 * a2 + 13.0 / 3.0 * a3 * a3;
    double t1 = b2 + b4 / 10.0, t2 = b3 + 123.0 / 455.0 * b5;
    double beta3 = t1 * t1 + 13.0 / 3.0 * t2 * t2 + 781.0 / 20.0 * b4 * b4
                 + 1421461.0 / 2275.0 * b5 * b5;
    double tau = (fabs(beta3 - beta1) + fabs(beta3 - beta2)) / 2.0;
    tau = tau * tau;
    double wb1 = chi[0] * (1.0 + tau / (eps + beta1));
    double wb2 = chi[1] * (1.0 + tau / (eps + beta2));
    double wb3 = chi[2] * (1.0 + tau / (eps + beta3));
    double sw = wb1 + wb2 + wb3;
    double w1 = wb1 / sw, w2 = wb2 / sw, w3 = wb3 / sw;

    /* Legendre basis at xi_{j+1/2}: L1 = 1, L2 = 1/2, L3 = 1/4 - 1/12,
       L4 = 1/8 - 3/40, L5 = 1/16 - 3/56 + 3/560 */
    double L2 = 0.5, L3 = 0.25 - 1.0 / 12.0, L4 = 0.125 - 3.0 / 40.0;
    double L5 = 1.0 / 16.0 - 3.0 / 56.0 + 3.0 / 560.0;
    double h1 = W0;
    double h2 = a1 + a2 * L2 + a3 * L3;
    double h3 = b1 + b2 * L2 + b3 * L3 + b4 * L4 + b5 * L5;
    return w1 * h1 + w2 * h2
         + w3 * (h3 / chi[2] - chi[0] / chi[2] * h1 - chi[1] / chi[2] * h2);
}

/* ------------------------------------------------------------------------ */
/* The paper's comparison variant MM-WENOJS (Section 5) swaps the MR         */
/* reconstruction for the classical fifth-order WENO of Jiang and Shu, cited */
/* there.  Written from its published definition: the three third-order     */
/* candidates on the sub-stencils {i-2..i}, {i-1..i+1}, {i..i+2} at the     */
/* right face of node i, the smoothness indicators beta_k, and the weights   */
/* alpha_k = d_k / (eps + beta_k)^2 normalised, d = (1/10, 6/10, 3/10).      */
/* ------------------------------------------------------------------------ */
double orc_js5(const double *q, double eps)
{
    double qm2 = q[0], qm1 = q[1], q0 = q[2], qp1 = q[3], qp2 = q[4];
    double c[3], beta[3], alpha[3];
    const double d[3] = {0.1, 0.6, 0.3};
    c[0] = (2.0 * qm2 - 7.0 * qm1 + 11.0 * q0) / 6.0;
    c[1] = (-qm1 + 5.0 * q0 + 2.0 * qp1) / 6.0;
    c[2] = (2.0 * q0 + 5.0 * qp1 - qp2) / 6.0;
    beta[0] = 13.0 / 12.0 * (qm2 - 2.0 * qm1 + q0) * (qm2 - 2.0 * qm1 + q0)
            + 0.25 * (qm2 - 4.0 * qm1 + 3.0 * q0) * (qm2 - 4.0 * qm1 + 3.0 * q0);
    beta[1] = 13.0 / 12.0 * (qm1 - 2.0 * q0 + qp1) * (qm1 - 2.0 * q0 + qp1)
            + 0.25 * (qm1 - qp1) * (qm1 - qp1);
    beta[2] = 13.0 / 12.0 * (q0 - 2.0 * qp1 + qp2) * (q0 - 2.0 * qp1 + qp2)
            + 0.25 * (3.0 * q0 - 4.0 * qp1 + qp2) * (3.0 * q0 - 4.0 * qp1 + qp2);
    double sa = 0.0;
    for (int k = 0; k < 3; k++) {
        alpha[k] = d[k] / ((eps + beta[k]) * (eps + beta[k]));
        sa += alpha[k];
    }
    double v = 0.0;
    for (int k = 0; k < 3; k++) v += alpha[k] / sa * c[k];
    return v;
}

/* ------------------------------------------------------------------------ */
/* ghost layers                                                             */
/* Periodic directions wrap.  The paper names the boundary conditions of    */
/* its examples (periodic; reflecting, inflow and outflow for the shock-    */
/* bubble runs) without their discrete form.  Reading used here: nodes are  */
/* cell-centred, so the face of a non-periodic direction lies halfway       */
/* between the outermost interior node and the first ghost node, and the    */
/* ghost node m layers outside the face images the interior node m - 1      */
/* layers inside it (a mirror).  On such a face                             */
/*   - the mesh is mirrored about the face's physical coordinate wall:      */
/*     x_k -> 2 wall - x_k, the other coordinates kept (for every kind of   */
/*     non-periodic face), so the Jacobi sweeps keep the face in place and  */
/*     let the nodes next to it slide along it;                             */
/*   - fields without a direction (J, monitor values) are mirrored copies;  */
/*   - displacements are mirrored with component k negated, metrics         */
/*     J dxi_a/dx_b mirrored and negated when exactly one of a, b is k,     */
/*     J dxi_a/dt negated when a = k (what the mirrored mesh gives);        */
/*   - the state: a reflecting wall mirrors U with the momentum component   */
/*     k negated; outflow copies U of the outermost interior node; inflow   */
/*     takes the face's prescribed state; JU = J (mirrored) times that U.   */
/* Every out-of-range coordinate of a ghost node is mapped at once (edges   */
/* and corners compose the rules of their directions; where an inflow face */
/* is involved, the inflow state of the lowest such direction is taken).    */
/* ------------------------------------------------------------------------ */
enum { BC_PERIODIC = 0, BC_REFLECT = 1, BC_OUTFLOW = 2, BC_INFLOW = 3 };
enum { GH_PLAIN = 0, GH_MESH = 1, GH_DISP = 2, GH_JXX = 3, GH_JXT = 4 };

/* image of padded index i along direction k: *side = -1 below, +1 above,
   0 inside; *kind = the face's condition (periodic or not) */
static int image(const orc_grid *g, int k, int i, int *side, int *kind)
{
    int n = g->n[k], ng = g->ng, r = i - ng;
    *side = r < 0 ? -1 : (r >= n ? 1 : 0);
    *kind = *side ? g->bc[k][*side > 0] : -1;
    if (!*side) return i;
    if (*kind == BC_PERIODIC) return (*side < 0 ? r + n : r - n) + ng;
    return (*side < 0 ? -1 - r : 2 * n - 1 - r) + ng;
}

static void fill_ghosts_impl(const orc_grid *g, double *a, int ncomp, int what)
{
    long P = orc_npoints(g);
    int d = g->dim;
    for (int i2 = 0; i2 < npad(g, 2); i2++)
        for (int i1 = 0; i1 < npad(g, 1); i1++)
            for (int i0 = 0; i0 < npad(g, 0); i0++) {
                int idx[3] = {i0, i1, i2}, src[3] = {i0, i1, i2}, side[3] = {0, 0, 0};
                int kind[3] = {-1, -1, -1}, ghost = 0;
                for (int k = 0; k < d; k++) {
                    src[k] = image(g, k, idx[k], &side[k], &kind[k]);
                    if (side[k]) ghost = 1;
                }
                if (!ghost) continue;
                long dst = at(g, i0, i1, i2), from = at(g, src[0], src[1], src[2]);
                for (int c = 0; c < ncomp; c++) {
                    double v = a[c * P + from];
                    for (int k = 0; k < d; k++) {
                        if (!side[k]) continue;
                        if (kind[k] == BC_PERIODIC) {
                            /* component k of x carries +-L_k when wrapped along k */
                            if (what == GH_MESH && c == k) v += side[k] * g->len[k];
                            continue;
                        }
                        if (what == GH_MESH && c == k) v = 2.0 * g->wall[k][side[k] > 0] - v;
                        if ((what == GH_DISP || what == GH_JXT) && c == k) v = -v;
                        if (what == GH_JXX && ((c / d == k) != (c % d == k))) v = -v;
                    }
                    a[c * P + dst] = v;
                }
            }
}

void orc_fill_ghosts(const orc_grid *g, double *a, int ncomp) { fill_ghosts_impl(g, a, ncomp, GH_PLAIN); }
void orc_fill_ghosts_x(const orc_grid *g, double *x) { fill_ghosts_impl(g, x, g->dim, GH_MESH); }
void orc_fill_ghosts_kind(const orc_grid *g, double *a, int ncomp, int what)
{
    fill_ghosts_impl(g, a, ncomp, what);
}

/* the state (JU, J): J first (mirrored or wrapped), then JU by the rules
   above */
void orc_fill_ghosts_state(const orc_grid *g, double *JU, double *J)
{
    long P = orc_npoints(g);
    int d = g->dim, N = g->nspec, nc = orc_ncomp(g);
    orc_fill_ghosts(g, J, 1);
    for (int i2 = 0; i2 < npad(g, 2); i2++)
        for (int i1 = 0; i1 < npad(g, 1); i1++)
            for (int i0 = 0; i0 < npad(g, 0); i0++) {
                int idx[3] = {i0, i1, i2}, src[3] = {i0, i1, i2};
                int ghost = 0, extrap = 0, flip[3] = {0, 0, 0};
                const double *uin = NULL;
                for (int k = 0; k < d; k++) {
                    int side, kind;
                    src[k] = image(g, k, idx[k], &side, &kind);
                    if (!side) continue;
                    ghost = 1;
                    if (kind == BC_REFLECT) flip[k] = 1;
                    if (kind == BC_OUTFLOW) {
                        src[k] = side < 0 ? g->ng : g->ng + g->n[k] - 1;
                        extrap = 1;
                    }
                    if (kind == BC_INFLOW && !uin) uin = g->inflow[k][side > 0];
                }
                if (!ghost) continue;
                long dst = at(g, i0, i1, i2), from = at(g, src[0], src[1], src[2]);
                double U[8];
                for (int c = 0; c < nc; c++) {
                    if (uin) U[c] = J[dst] * uin[c];
                    else if (extrap) U[c] = J[dst] * (JU[c * P + from] / J[from]);
                    else U[c] = JU[c * P + from];
                }
                if (!uin)
                    for (int k = 0; k < d; k++)
                        if (flip[k]) U[N + k] = -U[N + k];
                for (int c = 0; c < nc; c++) JU[c * P + dst] = U[c];
            }
}

/* ------------------------------------------------------------------------ */
/* Section 3.2, discrete GCL metrics.                                       */
/* delta_k[a]_i = 1/2 sum_m alpha_{w,m} (a_{i,k,+m} - a_{i,k,-m})            */
/* 3D (eq SCLCoeff, extended cyclically in j): with (k,a,b) and (j,p,q)      */
/* cyclic permutations of (1,2,3),                                           */
/*   J dxi_k/dx_j = (delta_b[delta_a[x_p] x_q] - delta_a[delta_b[x_p] x_q])  */
/*                  / (dxi_a dxi_b).                                        */
/* 2D (degenerate case): J dxi_1/dx = (delta_2 x_2, -delta_2 x_1)/dxi_2,     */
/*                       J dxi_2/dx = (-delta_1 x_2, delta_1 x_1)/dxi_1.     */
/* VCL (eq VCLCoeff): J dxi_k/dt = -sum_j xdot_j J dxi_k/dx_j with           */
/* xdot = disp / dt; the stage mesh is x = x^n + c_s disp.                  */
/* ------------------------------------------------------------------------ */
static double delta_k(const orc_grid *g, const double *a, long i, int k)
{
    double al[3];
    orc_alpha(g->w, al);
    long st = stride_(g, k);
    double s = 0.0;
    for (int m = 1; m <= g->w; m++) s += al[m - 1] * (a[i + m * st] - a[i - m * st]);
    return 0.5 * s;
}

/* delta_b[ delta_a[x_p] * x_q ] at node i; xs = stage mesh (dim components) */
static double nested(const orc_grid *g, const double *xs, long i, int a, int b, int p, int q)
{
    double al[3];
    orc_alpha(g->w, al);
    long P = orc_npoints(g), st = stride_(g, b);
    double s = 0.0;
    for (int m = 1; m <= g->w; m++) {
        long ip = i + m * st, im = i - m * st;
        double fp = delta_k(g, xs + p * P, ip, a) * xs[q * P + ip];
        double fm = delta_k(g, xs + p * P, im, a) * xs[q * P + im];
        s += al[m - 1] * (fp - fm);
    }
    return 0.5 * s;
}

/* Discrete Jacobian of the mesh (Section 3.2: J is the determinant of the  */
/* Jacobian matrix dx/dxi, whose cofactor rows are the metrics J dxi_k/dx):  */
/* by the cofactor expansion along each column k, det = sum_j dx_j/dxi_k     */
/* J dxi_k/dx_j; reading: dx_j/dxi_k by the same 2w-order difference as the  */
/* metrics, averaged over k.  Used only to set J on a non-uniform mesh at    */
/* t = 0; afterwards J follows eq semi_J.                                   */
int orc_jacobian(const orc_grid *g, const double *x, const double *jxi_x, double *J)
{
    if (!valid_grid(g) || !x || !jxi_x || !J) return ORC_EINVAL;
    int d = g->dim;
    long P = orc_npoints(g);
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double s = 0.0;
                for (int k = 0; k < d; k++)
                    for (int j = 0; j < d; j++)
                        s += delta_k(g, x + j * P, i, k) / g->dxi[k] * jxi_x[(k * d + j) * P + i];
                J[i] = s / d;
            }
    orc_fill_ghosts(g, J, 1);
    return ORC_OK;
}

int orc_metrics(const orc_grid *g, const double *x_n, const double *disp,
                double c_s, double dt, double *jxi_x, double *jxi_t)
{
    if (!valid_grid(g) || !x_n || !jxi_x) return ORC_EINVAL;
    int d = g->dim;
    long P = orc_npoints(g);
    double *xs = (double *)malloc((size_t)d * P * sizeof(double));
    if (!xs) return ORC_EINVAL;
    for (long t = 0; t < d * P; t++) xs[t] = x_n[t] + (disp ? c_s * disp[t] : 0.0);

#pragma omp parallel for collapse(2) schedule(static)
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double M[3][3];
                if (d == 2) {
                    M[0][0] = delta_k(g, xs + 1 * P, i, 1) / g->dxi[1];
                    M[0][1] = -delta_k(g, xs + 0 * P, i, 1) / g->dxi[1];
                    M[1][0] = -delta_k(g, xs + 1 * P, i, 0) / g->dxi[0];
                    M[1][1] = delta_k(g, xs + 0 * P, i, 0) / g->dxi[0];
                } else {
                    for (int k = 0; k < 3; k++) {
                        int a = (k + 1) % 3, b = (k + 2) % 3;
                        for (int j = 0; j < 3; j++) {
                            int p = (j + 1) % 3, q = (j + 2) % 3;
                            M[k][j] = (nested(g, xs, i, a, b, p, q) - nested(g, xs, i, b, a, p, q))
                                    / (g->dxi[a] * g->dxi[b]);
                        }
                    }
                }
                for (int k = 0; k < d; k++)
                    for (int j = 0; j < d; j++) jxi_x[(k * d + j) * P + i] = M[k][j];
                if (jxi_t) {
                    for (int k = 0; k < d; k++) {
                        double nt = 0.0;
                        if (disp && dt > 0.0)
                            for (int j = 0; j < d; j++) nt -= (disp[j * P + i] / dt) * M[k][j];
                        jxi_t[k * P + i] = nt;
                    }
                }
            }
    free(xs);
    orc_fill_ghosts_kind(g, jxi_x, d * d, GH_JXX);
    if (jxi_t) orc_fill_ghosts_kind(g, jxi_t, d, GH_JXT);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sections 3.1-3.4: interface flux at {i,k,+1/2}.                          */
/* EC part (eq ECFlux_curv_2p, eq GCL_flux):                                */
/*   F = sum_m alpha_{w,m} sum_{s=0}^{m-1} Fhat(U_{i-s}, U_{i-s+m}, ...),    */
/*   G = sum_m alpha_{w,m} sum_{s=0}^{m-1} 1/2 (n_t,{i-s} + n_t,{i-s+m}).    */
/* ES part (eq HOstable): F -= 1/2 T^T R s Y [[W]]^WENO.                     */
/* Readings: interface metrics nbar = (m_i + m_{i+1})/2 for the dissipation; */
/* W_j = R^T T V(U_j) for j = i-2..i+3 with R, T frozen at the interface;    */
/* W^+ is MR5 of the mirrored sequence W_{i+3..i-1}; Y_mm = 1 only if        */
/* [[W_m]]^WENO [[W_m]] > 0 and |[[W_m]]| > sign_tol B_m (sign_tol = 0: the  */
/* paper's rule as printed).                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_grid *g;
    const double *JU, *J, *jxi_x, *jxi_t;
    long P;
} fields_t;

/* what the sign test saw at one interface (orc_sign_test), and the term
   magnitudes of the interface flux (orc_mixed_bound) */
typedef struct {
    double jump[MAXC], jw[MAXC], bound[MAXC], s;
    int Y[MAXC];
    double ecmag[MAXC];          /* sum_m |alpha_m| sum_s |terms| of the pair fluxes */
    double w6[MAXC];             /* sum over the six stencil nodes of sum_e |R_ec| |(T V)_e| */
    double hsTR[MAXC * MAXC];    /* 1/2 s |(T^T R)_cm| */
} sign_info_t;

/* Bound on the size of the terms that form W_c at nodes i and i+1.  With
 * row magnitudes a_l = |V_l| (species), a_{N+j} = sum_j' |V_{N+j'}| (every
 * momentum row: an orthogonal T gives |(T V)_{N+j}| <= ||V_mom||_2 <=
 * ||V_mom||_1) and a_E = |V_E|, each summed over the two nodes,
 *   B_c = max_l |R_lc| sum_l a_l + sum_{e >= N} |R_ec| a_e
 *      >= sum_e |R_ec| (|(T V_i)_e| + |(T V_{i+1})_e|).
 * Forming W_c and the difference W_c(i+1) - W_c(i) rounds each of those
 * terms, so a jump of a few ulps of B_c is not resolved by the arithmetic. */
static void sign_bound_of(const orc_grid *g, const double *Vl, const double *Vr,
                          const double *R, double *B)
{
    int N = g->nspec, d = g->dim, nc = N + d + 1;
    double arow[MAXC];
    for (int e = 0; e < nc; e++) arow[e] = 0.0;
    const double *V2[2] = {Vl, Vr};
    for (int t = 0; t < 2; t++) {
        const double *V = V2[t];
        double vm = 0.0;
        for (int j = 0; j < d; j++) vm += fabs(V[N + j]);
        for (int l = 0; l < N; l++) arow[l] += fabs(V[l]);
        for (int a = 0; a < d; a++) arow[N + a] += vm;
        arow[nc - 1] += fabs(V[nc - 1]);
    }
    double ysum = 0.0;
    for (int l = 0; l < N; l++) ysum += arow[l];
    for (int c = 0; c < nc; c++) {
        double rmax = 0.0;
        for (int l = 0; l < N; l++) if (fabs(R[l * nc + c]) > rmax) rmax = fabs(R[l * nc + c]);
        B[c] = rmax * ysum;
        for (int e = N; e < nc; e++) B[c] += fabs(R[e * nc + c]) * arow[e];
    }
}

static int node_load(const fields_t *f, long i, int k, double *U, prim_t *q, double *m)
{
    const orc_grid *g = f->g;
    int d = g->dim, nc = orc_ncomp(g);
    double Jv = f->J[i];
    for (int c = 0; c < nc; c++) U[c] = f->JU[c * f->P + i] / Jv;
    m[0] = f->jxi_t ? f->jxi_t[k * f->P + i] : 0.0;
    for (int j = 0; j < d; j++) m[1 + j] = f->jxi_x[(k * d + j) * f->P + i];
    int rc = prim_of(g, U, q);
    if (!(Jv > 0.0)) rc = ORC_ETANGLE;
    return rc;
}

static int interface_flux(const fields_t *f, long i, int k, double *F, double *G, double *prod,
                          sign_info_t *info)
{
    const orc_grid *g = f->g;
    int N = g->nspec, d = g->dim, nc = N + d + 1;
    long st = stride_(g, k);
    double U[6][MAXC], M[6][4];
    prim_t q[6];
    int rc = ORC_OK;
    for (int t = 0; t < 6; t++) {          /* nodes i-2 .. i+3 */
        int r = node_load(f, i + (t - 2) * st, k, U[t], &q[t], M[t]);
        if (r && !rc) rc = r;
    }
    if (rc) return rc;

    double al[3];
    orc_alpha(g->w, al);
    for (int c = 0; c < nc; c++) F[c] = 0.0;
    *G = 0.0;
    if (info) memset(info, 0, sizeof(*info));
    for (int m = 1; m <= g->w; m++)
        for (int s = 0; s < m; s++) {
            int a = 2 - s, b = 2 - s + m;   /* slots of nodes i-s and i-s+m */
            double Fh[MAXC];
            ec_flux_of(g, &q[a], &q[b], M[a], M[b], Fh);
            for (int c = 0; c < nc; c++) F[c] += al[m - 1] * Fh[c];
            *G += al[m - 1] * 0.5 * (M[a][0] + M[b][0]);
            if (info) {
                double Fm[MAXC];
                ec_flux_mag_of(g, &q[a], &q[b], M[a], M[b], Fm);
                for (int c = 0; c < nc; c++) info->ecmag[c] += fabs(al[m - 1]) * Fm[c];
            }
        }
    if (prod) *prod = 0.0;
    if (!g->dissipation) return ORC_OK;

    double mbar[4];
    for (int t = 0; t < 4; t++) mbar[t] = 0.5 * (M[2][t] + M[3][t]);
    double R[MAXC * MAXC], s, Tv[3][3];
    frame_of(g, &q[2], &q[3], mbar, R, &s, Tv);

    double W[6][MAXC], Vi[MAXC], Vi1[MAXC], Wmag[MAXC];
    for (int t = 0; t < 6; t++) {
        double V[MAXC], TV[MAXC];
        entropy_vars_of(g, &q[t], V);
        if (t == 2) for (int c = 0; c < nc; c++) Vi[c] = V[c];
        if (t == 3) for (int c = 0; c < nc; c++) Vi1[c] = V[c];
        for (int c = 0; c < nc; c++) TV[c] = V[c];
        for (int a = 0; a < d; a++) {
            TV[N + a] = 0.0;
            for (int b = 0; b < d; b++) TV[N + a] += Tv[a][b] * V[N + b];
        }
        for (int c = 0; c < nc; c++) {
            W[t][c] = 0.0;
            for (int e = 0; e < nc; e++) W[t][c] += R[e * nc + c] * TV[e];   /* R^T */
            if (info)
                for (int e = 0; e < nc; e++) info->w6[c] += fabs(R[e * nc + c]) * fabs(TV[e]);
        }
    }
    sign_bound_of(g, Vi, Vi1, R, Wmag);
    double Z[MAXC], pr = 0.0;
    for (int c = 0; c < nc; c++) {
        double qm[5] = {W[0][c], W[1][c], W[2][c], W[3][c], W[4][c]};
        double qp[5] = {W[5][c], W[4][c], W[3][c], W[2][c], W[1][c]};
        double Wminus = g->reconstruction ? orc_js5(qm, g->weno_eps) : orc_mr5(qm, g->chi, g->weno_eps);
        double Wplus = g->reconstruction ? orc_js5(qp, g->weno_eps) : orc_mr5(qp, g->chi, g->weno_eps);
        double JW = Wplus - Wminus;
        double jump = W[3][c] - W[2][c];
        /* sign matrix: Y_mm = 1 iff the WENO jump and the jump agree in
           sign.  With sign_tol > 0, a jump no larger than sign_tol times
           the bound on the terms that form it (sign_bound_of) counts as
           zero, so Y_mm = 0 there: across a contact the acoustic jumps
           vanish up to rounding, in an isentropic flow the entropy field's
           do, and the sign of such a jump is decided by rounding order */
        int Y = (JW * jump > 0.0) && (fabs(jump) > g->sign_tol * Wmag[c]);
        Z[c] = Y ? JW : 0.0;
        if (Y) pr += 0.5 * s * jump * JW;
        if (info) {
            info->jump[c] = jump;
            info->jw[c] = JW;
            info->bound[c] = Wmag[c];
            info->Y[c] = Y;
        }
    }
    if (info) info->s = s;
    double RZ[MAXC], D[MAXC];
    for (int a = 0; a < nc; a++) {
        RZ[a] = 0.0;
        for (int b = 0; b < nc; b++) RZ[a] += R[a * nc + b] * Z[b];
    }
    for (int c = 0; c < nc; c++) D[c] = 0.5 * s * RZ[c];
    {   /* T^T on the velocity block */
        double tmp[3];
        for (int a = 0; a < d; a++) {
            tmp[a] = 0.0;
            for (int b = 0; b < d; b++) tmp[a] += Tv[b][a] * RZ[N + b];
        }
        for (int a = 0; a < d; a++) D[N + a] = 0.5 * s * tmp[a];
    }
    for (int c = 0; c < nc; c++) F[c] -= D[c];
    if (prod) *prod = pr;
    if (info) {   /* 1/2 s |T^T R| (T^T acts on the velocity rows) */
        for (int c = 0; c < nc; c++)
            for (int mm = 0; mm < nc; mm++) info->hsTR[c * nc + mm] = 0.5 * s * fabs(R[c * nc + mm]);
        for (int a = 0; a < d; a++)
            for (int mm = 0; mm < nc; mm++) {
                double t = 0.0;
                for (int b = 0; b < d; b++) t += Tv[b][a] * R[(N + b) * nc + mm];
                info->hsTR[(N + a) * nc + mm] = 0.5 * s * fabs(t);
            }
    }
    return ORC_OK;
}

int orc_sign_bound(const orc_grid *g, const double *Ul, const double *Ur,
                   const double *m, double *B)
{
    if (!valid_grid(g) || !Ul || !Ur || !m || !B) return ORC_EINVAL;
    prim_t l, r;
    int a = prim_of(g, Ul, &l), b = prim_of(g, Ur, &r);
    double R[MAXC * MAXC], s, Tv[3][3], Vl[MAXC], Vr[MAXC];
    frame_of(g, &l, &r, m, R, &s, Tv);
    entropy_vars_of(g, &l, Vl);
    entropy_vars_of(g, &r, Vr);
    sign_bound_of(g, Vl, Vr, R, B);
    return a ? a : b;
}

int orc_sign_test(const orc_grid *g, const double *JU, const double *J,
                  const double *jxi_x, const double *jxi_t, int k, int npts,
                  const long *pts, double *jump, double *jw, double *bound,
                  int *Y, double *s_out)
{
    if (!valid_grid(g) || !JU || !J || !jxi_x || k < 0 || k >= g->dim || npts < 0 || !pts ||
        !jump || !jw || !bound || !Y || !s_out || !g->dissipation)
        return ORC_EINVAL;
    fields_t f = {g, JU, J, jxi_x, jxi_t, orc_npoints(g)};
    int nc = orc_ncomp(g), rc = ORC_OK;
    for (int p = 0; p < npts; p++) {
        double F[MAXC], G;
        sign_info_t info;
        int r = interface_flux(&f, pts[p], k, F, &G, NULL, &info);
        if (r) {
            if (!rc) rc = r;
            continue;
        }
        for (int c = 0; c < nc; c++) {
            jump[p * nc + c] = info.jump[c];
            jw[p * nc + c] = info.jw[c];
            bound[p * nc + c] = info.bound[c];
            Y[p * nc + c] = info.Y[c];
        }
        s_out[p] = info.s;
    }
    return rc;
}

int orc_mixed_bound(const orc_grid *g, const double *JU, const double *J,
                    const double *jxi_x, const double *jxi_t, double kf, double kw,
                    double u, double tol32, int npts, const long *pts, double *bound)
{
    if (!valid_grid(g) || !JU || !J || !jxi_x || npts < 0 || !pts || !bound) return ORC_EINVAL;
    fields_t f = {g, JU, J, jxi_x, jxi_t, orc_npoints(g)};
    int nc = orc_ncomp(g), rc = ORC_OK;
    for (int p = 0; p < npts; p++) {
        double E[MAXC];
        for (int c = 0; c < nc; c++) E[c] = 0.0;
        for (int k = 0; k < g->dim; k++) {
            long st = stride_(g, k);
            for (int side = 0; side < 2; side++) {
                double F[MAXC], G;
                sign_info_t info;
                int r = interface_flux(&f, side ? pts[p] : pts[p] - st, k, F, &G, NULL, &info);
                if (r) { if (!rc) rc = r; continue; }
                for (int c = 0; c < nc; c++) {
                    double e = kf * u * info.ecmag[c];
                    if (g->dissipation)
                        for (int m = 0; m < nc; m++) {
                            double ajw = fabs(info.jw[m]);
                            int unresolved = fabs(info.jump[m]) <= (tol32 + kw * u) * info.bound[m];
                            e += info.hsTR[c * nc + m] *
                                 (kw * u * info.w6[m] + kf * u * ajw + (unresolved ? ajw : 0.0));
                        }
                    E[c] += e / g->dxi[k];
                }
            }
        }
        for (int c = 0; c < nc; c++) bound[p * nc + c] = E[c];
    }
    return rc;
}

/* eq semi_U, eq semi_J at one node */
static int node_rhs(const fields_t *f, long i, double *dU, double *dJ)
{
    const orc_grid *g = f->g;
    int nc = orc_ncomp(g);
    for (int c = 0; c < nc; c++) dU[c] = 0.0;
    *dJ = 0.0;
    for (int k = 0; k < g->dim; k++) {
        long st = stride_(g, k);
        double Fp[MAXC], Fm[MAXC], Gp, Gm;
        int r1 = interface_flux(f, i, k, Fp, &Gp, NULL, NULL);
        int r2 = interface_flux(f, i - st, k, Fm, &Gm, NULL, NULL);
        if (r1) return r1;
        if (r2) return r2;
        for (int c = 0; c < nc; c++) dU[c] -= (Fp[c] - Fm[c]) / g->dxi[k];
        *dJ -= (Gp - Gm) / g->dxi[k];
    }
    return ORC_OK;
}

int orc_rhs(const orc_grid *g, const double *JU, const double *J,
            const double *jxi_x, const double *jxi_t, double *dJU, double *dJ)
{
    if (!valid_grid(g) || !JU || !J || !jxi_x || !dJU || !dJ) return ORC_EINVAL;
    fields_t f = {g, JU, J, jxi_x, jxi_t, orc_npoints(g)};
    int nc = orc_ncomp(g), rc = ORC_OK;
    int n1 = hi_(g, 1) - lo_(g, 1), n2 = hi_(g, 2) - lo_(g, 2);
#pragma omp parallel for collapse(2) schedule(static)
    for (int i2 = lo_(g, 2); i2 < lo_(g, 2) + n2; i2++)
        for (int i1 = lo_(g, 1); i1 < lo_(g, 1) + n1; i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double dU[MAXC], dj;
                int r = node_rhs(&f, i, dU, &dj);
                if (r) {
#pragma omp critical
                    rc = r;
                }
                for (int c = 0; c < nc; c++) dJU[c * f.P + i] = dU[c];
                dJ[i] = dj;
            }
    return rc;
}

int orc_rhs_points(const orc_grid *g, const double *JU, const double *J,
                   const double *jxi_x, const double *jxi_t, int npts,
                   const long *pts, double *dJU, double *dJ)
{
    if (!valid_grid(g) || !JU || !J || !jxi_x || !pts || !dJU || !dJ) return ORC_EINVAL;
    fields_t f = {g, JU, J, jxi_x, jxi_t, orc_npoints(g)};
    int nc = orc_ncomp(g), rc = ORC_OK;
    for (int t = 0; t < npts; t++) {
        double dU[MAXC], dj;
        int r = node_rhs(&f, pts[t], dU, &dj);
        if (r && !rc) rc = r;
        for (int c = 0; c < nc; c++) dJU[(long)t * nc + c] = dU[c];
        dJ[t] = dj;
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Section 5, third-order SSP Runge-Kutta (Gottlieb, Shu & Tadmor) in        */
/* Shu-Osher form for Q = (JU, J):                                          */
/*   Q1 = Q^n + dt L(Q^n); Q2 = 3/4 Q^n + 1/4 (Q1 + dt L(Q1));                */
/*   Q^{n+1} = 1/3 Q^n + 2/3 (Q2 + dt L(Q2)).                                */
/* stage s: out = a_s Q^n + b_s (Q_s + dt L(Q_s)); c_s is the stage time    */
/* fraction (0, 1, 1/2) used for the stage mesh.                            */
/* ------------------------------------------------------------------------ */
void orc_rk_coeffs(int stage, double *a, double *b, double *c)
{
    static const double A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    static const double B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    static const double C[3] = {0.0, 1.0, 0.5};
    *a = A[stage]; *b = B[stage]; *c = C[stage];
}

int orc_rk_stage(const orc_grid *g, int stage, double dt,
                 const double *JU_n, const double *J_n,
                 const double *JU_s, const double *J_s,
                 const double *jxi_x, const double *jxi_t,
                 double *JU_out, double *J_out)
{
    if (!valid_grid(g) || stage < 0 || stage > 2) return ORC_EINVAL;
    long P = orc_npoints(g);
    int nc = orc_ncomp(g);
    double *L = (double *)calloc((size_t)(nc + 1) * P, sizeof(double));
    if (!L) return ORC_EINVAL;
    int rc = orc_rhs(g, JU_s, J_s, jxi_x, jxi_t, L, L + nc * P);
    double a, b, c;
    orc_rk_coeffs(stage, &a, &b, &c);
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                for (int cc = 0; cc < nc; cc++)
                    JU_out[cc * P + i] = a * JU_n[cc * P + i]
                                       + b * (JU_s[cc * P + i] + dt * L[cc * P + i]);
                J_out[i] = a * J_n[i] + b * (J_s[i] + dt * L[nc * P + i]);
            }
    free(L);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Section 5, CFL condition (eq cfl): dt = C / max_i sum_k rho_{i,k}/dxi_k,  */
/* rho_{i,k} the spectral radius in xi_k of the transformed system.          */
/* Reading: rho_{i,k} = (|v . n_k| + c |n_k|) / J_i with n_k = J dxi_k/dx at */
/* the current mesh and zero mesh velocity.                                 */
/* ------------------------------------------------------------------------ */
int orc_max_wavespeed(const orc_grid *g, const double *JU, const double *J,
                      const double *jxi_x, double cfl, double *lambda, double *dt)
{
    if (!valid_grid(g) || !JU || !J || !jxi_x) return ORC_EINVAL;
    long P = orc_npoints(g);
    int nc = orc_ncomp(g), d = g->dim, N = g->nspec, rc = ORC_OK;
    double lam = 0.0;
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double U[MAXC];
                prim_t q;
                for (int c = 0; c < nc; c++) U[c] = JU[c * P + i] / J[i];
                int r = prim_of(g, U, &q);
                if (r && !rc) rc = r;
                (void)N;
                double c = sqrt(mix_R(g, &q) * mix_gamma(g, &q) * q.T);
                double sum = 0.0;
                for (int k = 0; k < d; k++) {
                    double vn = 0.0, nn = 0.0;
                    for (int j = 0; j < d; j++) {
                        double n = jxi_x[(k * d + j) * P + i];
                        vn += q.v[j] * n;
                        nn += n * n;
                    }
                    sum += (fabs(vn) + c * sqrt(nn)) / J[i] / g->dxi[k];
                }
                if (sum > lam) lam = sum;
            }
    if (lambda) *lambda = lam;
    if (dt) *dt = cfl / lam;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Section 4, mesh redistribution.                                          */
/* Monitor (eq monitor): Theta = (1 + sum_k alpha_k (|grad sigma_k| /        */
/*   max |grad sigma_k|)^2)^(1/2).  Readings: grad_xi by second-order       */
/*   central differences; a term whose max is 0 is dropped.                 */
/* Form 1, the monitor of the isentropic-vortex examples (Section 5):       */
/*   Theta = (1 + sum_k alpha_k |grad sigma_k| / max |grad sigma_k|          */
/*   + beta_k |lap sigma_k| / max |lap sigma_k|)^(1/2), lap_xi by the        */
/*   second-order central difference sum_k (s_{i+e_k} - 2 s_i + s_{i-e_k})  */
/*   / dxi_k^2 (the same reading as grad_xi).                               */
/* Low-pass filter (Remark 4.1): Theta <- sum_{j in {0,+-1}^d}               */
/*   (1/2)^(|j|_1 + d) Theta_{i+j}, applied n_smooth times out of place.     */
/* Jacobi iteration: x^{[nu+1]}_i = sum_k (Theta_{k+1/2} x^{[nu]}_{i+e_k}    */
/*   + Theta_{k-1/2} x^{[nu]}_{i-e_k}) / dxi_k^2 over                       */
/*   sum_k (Theta_{k+1/2} + Theta_{k-1/2}) / dxi_k^2, exactly mu sweeps,     */
/*   Theta_{k+-1/2} = (Theta_i + Theta_{i+-e_k})/2.                          */
/* Limiter: Delta_tau = min(1, min over bounds), bound = -(x_k,i -           */
/*   x_k,i-e_k)/(2 dx_k) if dx_k < 0, (x_k,i+e_k - x_k,i)/(2 dx_k) if > 0.   */
/* disp = Delta_tau (x^{[mu]} - x^n); resid[nu] = max |x^{[nu+1]}-x^{[nu]}|. */
/* ------------------------------------------------------------------------ */
/* Monitor variables: 0 rho, 1 rho_1, 2 rho_2, 3 p, 4 |v| (the "u" of the   */
/*   multi-variable monitor of Example 5.9, read as the speed), 5 the        */
/*   schlieren function Phi = exp(-Psi |grad rho| / max |grad rho|) of eq    */
/*   schlieren with Psi = (psi_1 rho_1 + psi_2 rho_2) / rho (psi_1 alone for */
/*   one species), |grad rho| by the same central differences as the        */
/*   monitor, its max over the interior; Phi = 1 where that max is 0.  Phi  */
/*   is formed at the interior nodes and carried into the ghost layers like */
/*   any plain field.                                                        */
static double sigma_at(const orc_grid *g, const double *JU, const double *J, const double *phi,
                       long i, int sig)
{
    long P = orc_npoints(g);
    int nc = orc_ncomp(g);
    double U[MAXC];
    if (sig == 5) return phi[i];
    for (int c = 0; c < nc; c++) U[c] = JU[c * P + i] / J[i];
    if (sig == 0) { double r = 0.0; for (int l = 0; l < g->nspec; l++) r += U[l]; return r; }
    if (sig == 1) return U[0];
    if (sig == 2) return g->nspec > 1 ? U[1] : U[0];
    prim_t q;
    prim_of(g, U, &q);
    if (sig == 4) {
        double v2 = 0.0;
        for (int j = 0; j < g->dim; j++) v2 += q.v[j] * q.v[j];
        return sqrt(v2);
    }
    return q.p;
}

/* Phi at every interior node, ghost layers filled */
static void schlieren(const orc_grid *g, const orc_monitor *mo, const double *JU, const double *J,
                      double *phi);
int orc_schlieren(const orc_grid *g, const orc_monitor *mo, const double *JU, const double *J,
                  double *phi)
{
    if (!valid_grid(g) || !mo || !JU || !J || !phi) return ORC_EINVAL;
    schlieren(g, mo, JU, J, phi);
    return ORC_OK;
}

static void schlieren(const orc_grid *g, const orc_monitor *mo, const double *JU, const double *J,
                      double *phi)
{
    long P = orc_npoints(g);
    int d = g->dim;
    double *gr = (double *)calloc((size_t)P, sizeof(double));
    double gmax = 0.0;
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double g2 = 0.0;
                for (int k = 0; k < d; k++) {
                    long st = stride_(g, k);
                    double dk = (sigma_at(g, JU, J, NULL, i + st, 0) - sigma_at(g, JU, J, NULL, i - st, 0))
                                / (2.0 * g->dxi[k]);
                    g2 += dk * dk;
                }
                gr[i] = sqrt(g2);
                if (gr[i] > gmax) gmax = gr[i];
            }
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double r1 = sigma_at(g, JU, J, NULL, i, 1), rho = sigma_at(g, JU, J, NULL, i, 0);
                double psi = g->nspec > 1 ? (mo->psi[0] * r1 + mo->psi[1] * (rho - r1)) / rho : mo->psi[0];
                phi[i] = gmax > 0.0 ? exp(-psi * gr[i] / gmax) : 1.0;
            }
    free(gr);
    orc_fill_ghosts(g, phi, 1);
}

static void filter_pass(const orc_grid *g, const double *in, double *out)
{
    int d = g->dim;
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                double s = 0.0;
                int r2 = d == 3 ? 1 : 0;
                for (int j2 = -r2; j2 <= r2; j2++)
                    for (int j1 = -1; j1 <= 1; j1++)
                        for (int j0 = -1; j0 <= 1; j0++) {
                            int e = abs(j0) + abs(j1) + abs(j2) + d;
                            s += ldexp(1.0, -e) * in[at(g, i0 + j0, i1 + j1, i2 + j2)];
                        }
                out[at(g, i0, i1, i2)] = s;
            }
    orc_fill_ghosts(g, out, 1);
}

int orc_monitor_fn(const orc_grid *g, const orc_monitor *mo, const double *JU,
                   const double *J, double *theta)
{
    if (!valid_grid(g) || !mo || mo->nsig < 1 || mo->nsig > 6) return ORC_EINVAL;
    if (mo->form != 0 && (mo->form != 1 || mo->nsig > 2)) return ORC_EINVAL;
    long P = orc_npoints(g);
    int d = g->dim, use_phi = 0;
    for (int s = 0; s < mo->nsig; s++) {
        if (mo->sigma[s] < 0 || mo->sigma[s] > 5) return ORC_EINVAL;
        if (mo->sigma[s] == 5) use_phi = 1;
    }
    double *phi = NULL;
    if (use_phi) {
        phi = (double *)calloc((size_t)P, sizeof(double));
        schlieren(g, mo, JU, J, phi);
    }
    double *grad = (double *)calloc((size_t)mo->nsig * P, sizeof(double));
    double *lap = (double *)calloc((size_t)mo->nsig * P, sizeof(double));
    double gmax[6] = {0, 0, 0, 0, 0, 0}, lmax[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < mo->nsig; s++)
        for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
            for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
                for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                    long i = at(g, i0, i1, i2);
                    double g2 = 0.0;
                    for (int k = 0; k < d; k++) {
                        long st = stride_(g, k);
                        double dsk = (sigma_at(g, JU, J, phi, i + st, mo->sigma[s])
                                      - sigma_at(g, JU, J, phi, i - st, mo->sigma[s])) / (2.0 * g->dxi[k]);
                        g2 += dsk * dsk;
                    }
                    grad[s * P + i] = sqrt(g2);
                    if (grad[s * P + i] > gmax[s]) gmax[s] = grad[s * P + i];
                    if (mo->form == 1) {
                        double sc = sigma_at(g, JU, J, phi, i, mo->sigma[s]), l = 0.0;
                        for (int k = 0; k < d; k++) {
                            long st = stride_(g, k);
                            l += (sigma_at(g, JU, J, phi, i + st, mo->sigma[s]) - 2.0 * sc
                                  + sigma_at(g, JU, J, phi, i - st, mo->sigma[s])) / (g->dxi[k] * g->dxi[k]);
                        }
                        lap[s * P + i] = fabs(l);
                        if (lap[s * P + i] > lmax[s]) lmax[s] = lap[s * P + i];
                    }
                }
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double th = 1.0;
                for (int s = 0; s < mo->nsig; s++) {
                    if (gmax[s] > 0.0) {
                        double r = grad[s * P + i] / gmax[s];
                        th += mo->form == 1 ? mo->alpha[s] * r : mo->alpha[s] * r * r;
                    }
                    if (mo->form == 1 && lmax[s] > 0.0) th += mo->beta[s] * (lap[s * P + i] / lmax[s]);
                }
                theta[i] = sqrt(th);
            }
    free(grad);
    free(lap);
    free(phi);
    orc_fill_ghosts(g, theta, 1);
    double *tmp = (double *)calloc(P, sizeof(double));
    for (int s = 0; s < mo->n_smooth; s++) {
        filter_pass(g, theta, tmp);
        memcpy(theta, tmp, (size_t)P * sizeof(double));
    }
    free(tmp);
    return ORC_OK;
}

int orc_mesh_redistribute(const orc_grid *g, const orc_monitor *mo,
                          const double *JU, const double *J, const double *x_n,
                          double *disp, double *dtau, double *resid)
{
    if (!valid_grid(g) || !mo || !JU || !J || !x_n || !disp) return ORC_EINVAL;
    long P = orc_npoints(g);
    int d = g->dim;
    double *th = (double *)calloc(P, sizeof(double));
    double *xa = (double *)malloc((size_t)d * P * sizeof(double));
    double *xb = (double *)malloc((size_t)d * P * sizeof(double));
    int rc = orc_monitor_fn(g, mo, JU, J, th);
    memcpy(xa, x_n, (size_t)d * P * sizeof(double));
    for (int nu = 0; nu < mo->n_sweeps; nu++) {
        double r = 0.0;
        for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
            for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
                for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                    long i = at(g, i0, i1, i2);
                    for (int c = 0; c < d; c++) {
                        double num = 0.0, den = 0.0;
                        for (int k = 0; k < d; k++) {
                            long st = stride_(g, k);
                            double tp = 0.5 * (th[i] + th[i + st]);
                            double tm = 0.5 * (th[i] + th[i - st]);
                            double h2 = g->dxi[k] * g->dxi[k];
                            num += (tp * xa[c * P + i + st] + tm * xa[c * P + i - st]) / h2;
                            den += (tp + tm) / h2;
                        }
                        xb[c * P + i] = num / den;
                        double dd = fabs(xb[c * P + i] - xa[c * P + i]);
                        if (dd > r) r = dd;
                    }
                }
        orc_fill_ghosts_x(g, xb);
        if (resid) resid[nu] = r;
        double *t = xa; xa = xb; xb = t;
    }
    double dt = 1.0;
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                for (int k = 0; k < d; k++) {
                    long st = stride_(g, k);
                    double dx = xa[k * P + i] - x_n[k * P + i];
                    double b;
                    if (dx < 0.0) b = -(x_n[k * P + i] - x_n[k * P + i - st]) / (2.0 * dx);
                    else if (dx > 0.0) b = (x_n[k * P + i + st] - x_n[k * P + i]) / (2.0 * dx);
                    else continue;
                    if (b < dt) dt = b;
                }
            }
    if (!(dt > 0.0)) rc = ORC_ETANGLE;
    for (long t = 0; t < d * P; t++) disp[t] = 0.0;
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                for (int c = 0; c < d; c++) disp[c * P + i] = dt * (xa[c * P + i] - x_n[c * P + i]);
            }
    orc_fill_ghosts_kind(g, disp, d, GH_DISP);
    if (dtau) *dtau = dt;
    free(th); free(xa); free(xb);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Section 5, discrete total entropy sum_i J_i eta(U_i) dxi_1..dxi_d, and    */
/* the entropy rate sum_i (V_i^T dJU_i - phi_i dJ_i) dV, which equals        */
/* d/dt sum_i J_i eta_i because d(J eta) = V^T d(JU) - phi dJ.              */
/* ------------------------------------------------------------------------ */
double orc_total_entropy(const orc_grid *g, const double *JU, const double *J)
{
    long P = orc_npoints(g);
    int nc = orc_ncomp(g);
    double s = 0.0;
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double U[MAXC];
                prim_t q;
                for (int c = 0; c < nc; c++) U[c] = JU[c * P + i] / J[i];
                prim_of(g, U, &q);
                s += J[i] * entropy_of(g, &q);
            }
    return s * cell_volume(g);
}

double orc_entropy_rate(const orc_grid *g, const double *JU, const double *J,
                        const double *dJU, const double *dJ)
{
    long P = orc_npoints(g);
    int nc = orc_ncomp(g);
    double s = 0.0;
    for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
        for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
            for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                long i = at(g, i0, i1, i2);
                double U[MAXC], V[MAXC];
                prim_t q;
                for (int c = 0; c < nc; c++) U[c] = JU[c * P + i] / J[i];
                prim_of(g, U, &q);
                entropy_vars_of(g, &q, V);
                double t = -potential_of(g, &q) * dJ[i];
                for (int c = 0; c < nc; c++) t += V[c] * dJU[c * P + i];
                s += t;
            }
    return s * cell_volume(g);
}

/* the dissipation's entropy production:                                    */
/*   -sum_k dV/dxi_k sum_{i+1/2} s/2 sum_m Y_mm [[W_m]] [[W_m]]^WENO <= 0    */
double orc_es_production(const orc_grid *g, const double *JU, const double *J,
                         const double *jxi_x, const double *jxi_t)
{
    fields_t f = {g, JU, J, jxi_x, jxi_t, orc_npoints(g)};
    double tot = 0.0, dv = cell_volume(g);
    for (int k = 0; k < g->dim; k++)
        for (int i2 = lo_(g, 2); i2 < hi_(g, 2); i2++)
            for (int i1 = lo_(g, 1); i1 < hi_(g, 1); i1++)
                for (int i0 = lo_(g, 0); i0 < hi_(g, 0); i0++) {
                    double F[MAXC], G, pr = 0.0;
                    interface_flux(&f, at(g, i0, i1, i2), k, F, &G, &pr, NULL);
                    tot -= pr * dv / g->dxi[k];
                }
    return tot;
}

/* ------------------------------------------------------------------------ */
/* One time step in the order of Sections 4-5: mesh redistribution at t^n,   */
/* dt from the CFL condition on x^n, xdot = disp/dt, then the three RK       */
/* stages on the stage meshes x^n + c_s disp, and x^{n+1} = x^n + disp.      */
/* dt_fixed > 0 overrides the CFL step (accuracy runs).                     */
/* ------------------------------------------------------------------------ */
int orc_step(const orc_grid *g, const orc_monitor *mo, double cfl, double dt_fixed,
             int move_mesh, double *JU, double *J, double *x, double *dt_out,
             double *dtau_out)
{
    if (!valid_grid(g) || !JU || !J || !x) return ORC_EINVAL;
    long P = orc_npoints(g);
    int nc = orc_ncomp(g), d = g->dim, rc = ORC_OK, r;
    double *disp = (double *)calloc((size_t)d * P, sizeof(double));
    double *jx = (double *)calloc((size_t)d * d * P, sizeof(double));
    double *jt = (double *)calloc((size_t)d * P, sizeof(double));
    double *JUn = (double *)malloc((size_t)nc * P * sizeof(double));
    double *Jn = (double *)malloc((size_t)P * sizeof(double));
    double *JUo = (double *)calloc((size_t)nc * P, sizeof(double));
    double *Jo = (double *)calloc((size_t)P, sizeof(double));
    orc_fill_ghosts_state(g, JU, J);
    orc_fill_ghosts_x(g, x);
    double dtau = 0.0;
    if (move_mesh && mo) {
        r = orc_mesh_redistribute(g, mo, JU, J, x, disp, &dtau, NULL);
        if (r && !rc) rc = r;
    }
    double dt = dt_fixed;
    orc_metrics(g, x, NULL, 0.0, 0.0, jx, NULL);
    if (!(dt > 0.0)) {
        r = orc_max_wavespeed(g, JU, J, jx, cfl, NULL, &dt);
        if (r && !rc) rc = r;
    }
    memcpy(JUn, JU, (size_t)nc * P * sizeof(double));
    memcpy(Jn, J, (size_t)P * sizeof(double));
    for (int s = 0; s < 3; s++) {
        double a, b, c;
        orc_rk_coeffs(s, &a, &b, &c);
        orc_metrics(g, x, disp, c, dt, jx, jt);
        r = orc_rk_stage(g, s, dt, JUn, Jn, JU, J, jx, jt, JUo, Jo);
        if (r && !rc) rc = r;
        orc_fill_ghosts_state(g, JUo, Jo);
        memcpy(JU, JUo, (size_t)nc * P * sizeof(double));
        memcpy(J, Jo, (size_t)P * sizeof(double));
    }
    for (long t = 0; t < d * P; t++) x[t] += disp[t];
    orc_fill_ghosts_x(g, x);
    if (dt_out) *dt_out = dt;
    if (dtau_out) *dtau_out = dtau;
    free(disp); free(jx); free(jt); free(JUn); free(Jn); free(JUo); free(Jo);
    return rc;
}
