/*
 * es_oracle.h -- plain CPU FP64 oracle for the entropy-stable adaptive
 * moving-mesh finite-difference scheme of Li, Duan & Tang (arXiv 2202.07989).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Conventions
 *   - Structured grid, cell-centred computational nodes, i fastest.
 *   - Every field array is padded with g->ng ghost layers in each active
 *     direction; padded extents np[k] = n[k] + 2 ng (k < dim), np[2] = 1 in 2D.
 *   - A field with C components stores component c at offset c * P,
 *     P = np[0] * np[1] * np[2].
 *   - State JU has nc = nspec + dim + 1 components
 *     (J rho_1..J rho_N, J rho v_1..J rho v_d, J E); J has one.
 *   - Spatial metrics jxi_x hold dim*dim components, component (k*dim + j) is
 *     J dxi_k/dx_j; time metrics jxi_t hold dim components (J dxi_k/dt).
 *   - The mesh x holds dim components (x_1..x_d).
 *   - All functions take host pointers and run synchronously.
 *
 * Pins: every function is checked by the CPU tests against what the paper
 * and the mathematics fix (identities, closed forms, exactness, symmetry,
 * convergence), except one reading that is parity unpinned: the averaged
 * interface state used to build R for two species when the left and right
 * states differ (the paper leaves Y_l, H and d_l of the average open).  Any
 * symmetric positive choice keeps the scheme entropy stable, so only the
 * agreement with the GPU path fixes it.
 *
 * Return codes: 0 ok, -1 invalid argument, -4 non-physical state
 * (rho_l <= 0, T <= 0 or non-finite), -5 tangled mesh (J <= 0 or Delta_tau <= 0).
 */
#ifndef ES_ORACLE_H
#define ES_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int dim;           /* d = 2 or 3                                          */
    int nspec;         /* N = 1 or 2                                          */
    int n[3];          /* interior nodes per direction (n[2] = 1 in 2D)       */
    int ng;            /* ghost layers (>= 3)                                  */
    double dxi[3];     /* computational spacings Delta xi_k                    */
    double len[3];     /* physical period lengths L_k (periodic x ghost rule)  */
    int w;             /* EC order 2w, w in {1,2,3}                            */
    double gamma[2];   /* Gamma_l                                              */
    double cv[2];      /* c_{v,l}                                              */
    double pinf[2];    /* p_{infty,l}                                          */
    double chi[3];     /* MR-WENO linear weights                               */
    double weno_eps;   /* MR-WENO epsilon                                      */
    int dissipation;   /* 0: EC scheme, 1: ES scheme                           */
    int reconstruction;/* 0: multi-resolution WENO (Appendix A), 1: classical  */
                       /*    fifth-order WENO of Jiang and Shu (MM-WENOJS)     */
    int bc[3][2];      /* per face ([k][0] low, [k][1] high): 0 periodic,      */
                       /*    1 reflecting wall, 2 outflow, 3 inflow; a         */
                       /*    direction is periodic on both faces or neither    */
    double wall[3][2]; /* physical coordinate x_k of each non-periodic face    */
    double inflow[3][2][6]; /* prescribed conserved state U of inflow faces    */
    double sign_tol;   /* zero tolerance of the sign matrix Y (Section 3.4,   */
                       /*    after eq HOstable): Y_mm = 1 iff the WENO jump   */
                       /*    and the jump [[W_m]] agree in sign and           */
                       /*    |[[W_m]]| > sign_tol * B_m (B_m: orc_sign_bound);*/
                       /*    0 is the paper's rule as printed; 0 <= tol < 1   */
} orc_grid;

typedef struct {
    int nsig;          /* number of monitor variables kappa (1..6)             */
    int sigma[6];      /* 0: rho, 1: rho_1, 2: rho_2, 3: p, 4: |v|, 5: the     */
                       /*    schlieren function Phi (eq schlieren)             */
    double alpha[6];   /* alpha_k                                              */
    int n_smooth;      /* low-pass filter passes                               */
    int n_sweeps;      /* Jacobi iterations mu                                 */
    int form;          /* 0: eq monitor; 1: the isentropic-vortex form with a  */
                       /*    Laplacian term (Section 5), at most two variables */
    double beta[6];    /* Laplacian weights of form 1                          */
    double psi[2];     /* Psi = (psi_1 rho_1 + psi_2 rho_2) / rho of Phi       */
} orc_monitor;

/* ---- pointwise pieces (exposed for the pins) ---------------------------- */
int    orc_ncomp(const orc_grid *g);
void   orc_alpha(int w, double alpha[3]);
double orc_logmean(double al, double ar);
int    orc_prim(const orc_grid *g, const double *U, double *rho, double *v,
                double *T, double *p);
int    orc_entropy_vars(const orc_grid *g, const double *U, double *V);
double orc_entropy(const orc_grid *g, const double *U);
double orc_potential(const orc_grid *g, const double *U);
double orc_sound_speed(const orc_grid *g, const double *U);
void   orc_phys_flux(const orc_grid *g, const double *U, int j, double *F);
/* two-point EC flux; ml, mr = (J dxi_k/dt, J dxi_k/dx_1..x_d) at l and r */
int    orc_ec_flux(const orc_grid *g, const double *Ul, const double *Ur,
                   const double *ml, const double *mr, double *F);
/* rotation matrix T (nc x nc, row-major) for an interface normal n (dim) */
void   orc_rotation(const orc_grid *g, const double *n, double *T);
/* interface frame: R (nc x nc, row-major) at the rotated averaged state of
 * (Ul, Ur) for the averaged metric m = (n_t, n_1..n_d); s = max |eigenvalue| */
int    orc_interface_frame(const orc_grid *g, const double *Ul, const double *Ur,
                           const double *m, double *R, double *s);
/* bound B (nc values) on the size of the terms that form W_i and W_{i+1}
 * (W = R^T T V at the interface of Ul, Ur with averaged metric m): for
 * field c, B_c = max_l |R_lc| sum_l a_l (species rows) + sum_e |R_ec| a_e
 * (momentum and energy rows), a_l = |V_l|, a_{N+j} = sum_j' |V_{N+j'}|,
 * a_E = |V_E|, each summed over both nodes.  Since |(T V)_{N+j}| <=
 * sum_j' |V_{N+j'}| for an orthogonal T, B_c >= sum_e |R_ec| (|(T V_i)_e| +
 * |(T V_{i+1})_e|), the magnitude scale of the rounding of [[W_c]]. */
int    orc_sign_bound(const orc_grid *g, const double *Ul, const double *Ur,
                      const double *m, double *B);
/* the sign test at the interfaces between node pts[p] and its right
 * neighbour along direction k (p = 0..npts-1): per field c (index p*nc + c)
 * the jump [[W_c]], the WENO jump [[W_c]]^WENO, the bound B_c and Y_cc
 * (1 or 0) under g->sign_tol; s_out (npts values) the interface speed s.
 * Returns 0, or the first nonzero code of a node's primitives. */
int    orc_sign_test(const orc_grid *g, const double *JU, const double *J,
                     const double *jxi_x, const double *jxi_t, int k, int npts,
                     const long *pts, double *jump, double *jw, double *bound,
                     int *Y, double *s_out);
/* a-priori bound on |lower-precision - FP64| of the right-hand side at the
 * nodes pts (npts * nc values), for arithmetic of unit roundoff u in the
 * pair fluxes, frame, projections and reconstructions (test infrastructure,
 * not a step of the scheme).  Per node i and component c, summed over the
 * directions k and the two interfaces f of the node along k, divided by
 * dxi_k:  kf u |EC|_c(f) + sum_m 1/2 s |(T^T R)_cm| (kw u W6_m + kf u
 * |[[W_m]]^WENO| + [|[[W_m]]| <= (tol32 + kw u) B_m] |[[W_m]]^WENO|), with
 * |EC|_c the absolute summands of the six pair fluxes weighted by
 * |alpha_m|, W6_m = sum over the six stencil nodes of sum_e |R_em| |(T V)_e|,
 * B_m the sign-test bound; the last term covers a sign test that the lower
 * precision cannot resolve against its tolerance tol32. */
int    orc_mixed_bound(const orc_grid *g, const double *JU, const double *J,
                       const double *jxi_x, const double *jxi_t, double kf, double kw,
                       double u, double tol32, int npts, const long *pts, double *bound);
double orc_mr5(const double *q, const double *chi, double eps);
/* classical fifth-order WENO (Jiang & Shu 1996) at the right face of q[2]
 * from q[0..4], linear weights (1/10, 6/10, 3/10), alpha_k = d_k/(eps+beta_k)^2 */
double orc_js5(const double *q, double eps);

/* ---- whole-grid steps ----------------------------------------------------- */
long   orc_npoints(const orc_grid *g);
/* ghost layers: periodic wrap, or the mirror rules of non-periodic faces
 * (plain fields, the mesh, and what = 2 displacements, 3 jxi_x, 4 jxi_t);
 * the state (JU, J) by the reflecting / outflow / inflow rules */
void   orc_fill_ghosts(const orc_grid *g, double *a, int ncomp);
void   orc_fill_ghosts_x(const orc_grid *g, double *x);
void   orc_fill_ghosts_kind(const orc_grid *g, double *a, int ncomp, int what);
void   orc_fill_ghosts_state(const orc_grid *g, double *JU, double *J);
int    orc_metrics(const orc_grid *g, const double *x_n, const double *disp,
                   double c_s, double dt, double *jxi_x, double *jxi_t);
/* discrete Jacobian of a mesh from its metrics (for J at t = 0 on a mesh
 * that is not uniform): J = (1/d) sum_k sum_j delta_k[x_j]/dxi_k J dxi_k/dx_j */
int    orc_jacobian(const orc_grid *g, const double *x, const double *jxi_x, double *J);
int    orc_rhs(const orc_grid *g, const double *JU, const double *J,
               const double *jxi_x, const double *jxi_t, double *dJU, double *dJ);
int    orc_rhs_points(const orc_grid *g, const double *JU, const double *J,
                      const double *jxi_x, const double *jxi_t, int npts,
                      const long *pts, double *dJU, double *dJ);
void   orc_rk_coeffs(int stage, double *a, double *b, double *c);
int    orc_rk_stage(const orc_grid *g, int stage, double dt,
                    const double *JU_n, const double *J_n,
                    const double *JU_s, const double *J_s,
                    const double *jxi_x, const double *jxi_t,
                    double *JU_out, double *J_out);
int    orc_max_wavespeed(const orc_grid *g, const double *JU, const double *J,
                         const double *jxi_x, double cfl, double *lambda,
                         double *dt);
/* monitor Theta after the n_smooth filter passes (the Theta the Jacobi sweeps use) */
/* the schlieren function Phi (monitor variable 5) at the interior nodes,
 * ghost layers filled */
int    orc_schlieren(const orc_grid *g, const orc_monitor *mo, const double *JU,
                     const double *J, double *phi);
int    orc_monitor_fn(const orc_grid *g, const orc_monitor *m, const double *JU,
                      const double *J, double *theta);
int    orc_mesh_redistribute(const orc_grid *g, const orc_monitor *m,
                             const double *JU, const double *J,
                             const double *x_n, double *disp, double *dtau,
                             double *resid);
double orc_total_entropy(const orc_grid *g, const double *JU, const double *J);
double orc_entropy_rate(const orc_grid *g, const double *JU, const double *J,
                        const double *dJU, const double *dJ);
double orc_es_production(const orc_grid *g, const double *JU, const double *J,
                         const double *jxi_x, const double *jxi_t);
int    orc_step(const orc_grid *g, const orc_monitor *m, double cfl,
                double dt_fixed, int move_mesh, double *JU, double *J,
                double *x, double *dt_out, double *dtau_out);

#ifdef __cplusplus
}
#endif
#endif
