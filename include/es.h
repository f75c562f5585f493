/*
 * es.h -- C-ABI of libes.so, the MI355X (gfx950) path of the entropy-stable
 * adaptive moving-mesh finite-difference scheme of Li, Duan & Tang,
 * arXiv 2202.07989, for 2D/3D one- and two-species compressible Euler with
 * the stiffened equation of state.
 *
 * Data layout (every array is caller-owned device memory, FP64, contiguous)
 *   - Structured grid of cell-centred computational nodes, i fastest.
 *   - Each field is padded by g->ng ghost layers in every active direction:
 *     np[k] = n[k] + 2 ng for k < dim, np[2] = 1 in 2D, P = np0*np1*np2.
 *   - A field with C components stores component c at offset c*P.
 *   - JU: nc = nspec + dim + 1 components (J rho_1..J rho_N, J rho v, J E);
 *     J: 1 component; x, disp: dim components (mesh x_1..x_d and a mesh
 *     displacement); jxi_x: dim*dim components, component k*dim + j is
 *     J dxi_k/dx_j; jxi_t: dim components, J dxi_k/dt.
 *   - Device scalars (dt, lambda, Delta_tau, entropy sums) are single FP64
 *     values in device memory so a step needs no host synchronisation.
 *   - Each direction is periodic, or bounded by two faces each with a
 *     reflecting wall, outflow or inflow condition (es_grid.bc); ghost
 *     layers are filled by es_fill_ghosts / es_fill_ghosts_x /
 *     es_fill_ghosts_state, and by the calls that produce a field.
 *
 * Streams: every call is asynchronous on the given hipStream_t (passed as
 * void*, NULL = default stream).  A context must not be used from two host
 * threads at once, and two calls on one context must not overlap on
 * different streams (they share its workspace).
 *
 * Errors: calls return ES_OK (0) or a negative code.  Argument errors are
 * reported synchronously before anything is launched (ES_EINVAL,
 * ES_EUNSUPPORTED); ES_EHIP reports a failed launch or allocation.  Data
 * errors found inside kernels set bits of a device status word that
 * es_status() returns (ES_ST_NONPHYS: rho_l <= 0, T <= 0 or a non-finite
 * state; ES_ST_TANGLE: J <= 0 or Delta_tau <= 0).  Nothing is clamped or
 * repaired.
 */
#ifndef ES_H
#define ES_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ES_OK = 0,
    ES_EINVAL = -1,        /* bad argument (null pointer, size, stage)        */
    ES_EUNSUPPORTED = -2,  /* dim not 2/3, nspec not 1/2, w not 1..3, ng < 3  */
    ES_EHIP = -3,          /* HIP launch or allocation failure                */
    ES_ENONPHYS = -4,      /* returned by es_status when ES_ST_NONPHYS is set */
    ES_ETANGLE = -5        /* returned by es_status when ES_ST_TANGLE is set  */
};

enum { ES_ST_NONPHYS = 1u, ES_ST_TANGLE = 2u };

enum { ES_FP64 = 0, ES_MIXED = 1 };

/* interface reconstruction of the scaled entropy variables (Section 3.4):
 * ES_WENO_MR, the multi-resolution WENO of Appendix A (MM-WENOMR), or
 * ES_WENO_JS, the classical fifth-order WENO of Jiang and Shu that Section 5
 * runs for comparison (MM-WENOJS; linear weights 1/10, 6/10, 3/10, weights
 * d_k / (weno_eps + beta_k)^2; chi is not used).  ES_WENO_JS is FP64 only:
 * with ES_MIXED, es_create and es_batch_create return ES_EUNSUPPORTED. */
enum { ES_WENO_MR = 0, ES_WENO_JS = 1 };

/* face conditions (es_grid.bc).  Section 5 runs its shock-bubble examples
 * with reflecting walls on two faces and outflow / inflow on the others
 * (Example 5.8) without giving their discrete form.  Here nodes stay
 * cell-centred: a face lies halfway between the outermost interior node and
 * the first ghost node, and the ghost node m layers outside images the
 * interior node m - 1 layers inside (a mirror).  On every non-periodic face
 * the mesh is mirrored about the face's coordinate wall (x_k -> 2 wall -
 * x_k), so the mesh equations keep the face fixed and move the nodes along
 * it; J and other plain fields are mirrored copies.  The state: ES_BC_REFLECT
 * mirrors U with momentum component k negated; ES_BC_OUTFLOW copies U of
 * the outermost interior node; ES_BC_INFLOW sets the face's prescribed
 * conserved state es_grid.inflow; each times the mirrored J.  A direction
 * is periodic on both faces or on neither.  Batches take periodic grids
 * only (ES_EUNSUPPORTED). */
enum { ES_BC_PERIODIC = 0, ES_BC_REFLECT = 1, ES_BC_OUTFLOW = 2, ES_BC_INFLOW = 3 };

typedef struct {
    int dim;           /* d = 2 or 3                                            */
    int nspec;         /* N = 1 or 2                                            */
    int n[3];          /* interior nodes per direction (>= ng); n[2] = 1 in 2D  */
    int ng;            /* ghost layers, >= 3                                    */
    double dxi[3];     /* computational spacings Delta xi_k (> 0)               */
    double len[3];     /* physical period lengths L_k used by es_fill_ghosts_x  */
    int w;             /* EC flux order 2w, w in {1, 2, 3}                      */
    double gamma[2];   /* Gamma_l > 1                                           */
    double cv[2];      /* c_{v,l} > 0                                           */
    double pinf[2];    /* p_{infty,l} >= 0                                      */
    double chi[3];     /* MR-WENO linear weights (positive, sum 1)              */
    double weno_eps;   /* MR-WENO epsilon                                       */
    int dissipation;   /* 0: entropy-conservative scheme, 1: entropy-stable     */
    int precision;     /* ES_FP64, or ES_MIXED: FP32 flux/WENO arithmetic with  */
                       /* FP64 log means, metrics, mesh and entropy sums        */
    int reconstruction;/* ES_WENO_MR or ES_WENO_JS (else ES_EUNSUPPORTED)       */
    int bc[3][2];      /* ES_BC_* of the low [k][0] and high [k][1] face of     */
                       /* direction k; zero (all periodic) by default           */
    double wall[3][2]; /* physical coordinate x_k of each non-periodic face     */
                       /* (wall[k][1] > wall[k][0])                             */
    double inflow[3][2][6]; /* conserved state U (rho_1..rho_N, rho v, E) of    */
                       /* each ES_BC_INFLOW face (finite)                       */
    double sign_tol;   /* zero tolerance of the sign matrix Y (Section 3.4,     */
                       /* after eq HOstable) in FP64 arithmetic, and           */
    double sign_tol32; /* in the FP32 arithmetic of ES_MIXED: Y_mm = 1 iff the  */
                       /* WENO jump and the jump [[W_m]] agree in sign and      */
                       /* |[[W_m]]| > tol * B_m, B_m a bound on the terms that  */
                       /* form W_m at the two nodes (B_m >= sum_e |R_em|        */
                       /* (|(T V_i)_e| + |(T V_i+1)_e|)).  0 is the paper's     */
                       /* rule as printed; 0 <= tol < 1 (else ES_EINVAL).  The  */
                       /* reading used for the paper's workloads is 1e-12 and  */
                       /* 1e-6: where a contact leaves the acoustic jumps at    */
                       /* rounding level, Y is then not decided by rounding    */
} es_grid;

typedef struct {
    int nsig;          /* number of monitor variables kappa, 1..6               */
    int sigma[6];      /* 0: rho, 1: rho_1, 2: rho_2, 3: p, 4: the speed |v|,   */
                       /* 5: the schlieren function Phi (below)                 */
    double alpha[6];   /* alpha_k >= 0                                          */
    int n_smooth;      /* low-pass filter passes                                */
    int n_sweeps;      /* Jacobi iterations mu (1..4096)                        */
    int form;          /* ES_MONITOR_GRAD2 or ES_MONITOR_GRAD_LAP (below)       */
    double beta[6];    /* Laplacian weights of ES_MONITOR_GRAD_LAP, >= 0        */
    double psi[2];     /* weights of Phi's Psi (finite)                         */
} es_monitor;

/* The monitor of Example 5.9 combines (Phi, u, rho_1, rho_2, p); u is taken
 * as the speed |v|.  Phi is the schlieren function of eq schlieren, Phi =
 * exp(-Psi |grad rho| / max |grad rho|), Psi = (psi[0] rho_1 + psi[1]
 * rho_2) / rho (psi[0] for one species), |grad rho| by the monitor's
 * central differences in xi, its maximum over the interior nodes (Phi = 1
 * where that maximum is 0); Phi is formed at the interior nodes and carried
 * into the ghost layers like a plain field. */

/* monitor forms: ES_MONITOR_GRAD2 is eq monitor, Theta = (1 + sum_k alpha_k
 * (|grad sigma_k| / max|grad sigma_k|)^2)^(1/2); ES_MONITOR_GRAD_LAP is the
 * form of the isentropic-vortex examples (Section 5), Theta = (1 + sum_k
 * alpha_k |grad sigma_k| / max|grad sigma_k| + beta_k |lap sigma_k| /
 * max|lap sigma_k|)^(1/2), at most two variables.  grad and lap are
 * second-order central differences in xi; a term whose maximum is 0 is
 * dropped. */
enum { ES_MONITOR_GRAD2 = 0, ES_MONITOR_GRAD_LAP = 1 };

typedef struct es_ctx es_ctx;

/* Create a context for one grid on the current device: validates g, then
 * allocates and initialises the whole workspace of the context (status word,
 * reduction scratch, the metric, mesh and stage buffers of es_step and the
 * kept-metrics copy): 67 P doubles in 3D with two species (9.6 GB at
 * 256^3).  This is the only call that allocates or synchronises the
 * device; every other call only launches work on its stream, so it may be
 * captured in a graph from its first use.  Owns only its workspace;
 * ES_EHIP when an allocation fails. */
int es_create(const es_grid *g, es_ctx **out);
int es_destroy(es_ctx *c);

/* Ghost layers of an ncomp-component field without direction (J, monitor
 * values): periodic copies, mirrored copies across non-periodic faces. */
int es_fill_ghosts(es_ctx *c, double *a, int ncomp, void *stream);

/* Ghost layers of the mesh x: component k gains +-L_k when wrapped along a
 * periodic direction k (x(xi + L e_k) = x(xi) + L_k e_k); mirrored about
 * the face (x_k -> 2 wall - x_k) across a non-periodic one. */
int es_fill_ghosts_x(es_ctx *c, double *x, void *stream);

/* Ghost layers of the state: J (as es_fill_ghosts), then JU by the face
 * conditions (ES_BC_*).  JU and J must differ (ES_EINVAL). */
int es_fill_ghosts_state(es_ctx *c, double *JU, double *J, void *stream);

/* Section 3.2, eq SCLCoeff / eq VCLCoeff: metrics of the stage mesh
 * x = x_n + c_s * disp (disp may be NULL: fixed mesh).  jxi_x gets the
 * 2w-th order conservative cross-derivative form at interior nodes; jxi_t =
 * -sum_j (disp_j / dt) jxi_x[k][j] when disp and dt_dev are given, else 0.
 * Ghost layers of the outputs are filled (wrapped, or as the mirrored mesh
 * gives them across non-periodic faces).  x_n and disp need
 * valid ghost layers.  flags: 0, or ES_METRICS_VCL_ONLY to recompute only
 * jxi_t from an existing jxi_x. */
enum { ES_METRICS_VCL_ONLY = 1 };
int es_metrics(es_ctx *c, const double *x_n, const double *disp, double c_s,
               const double *dt_dev, double *jxi_x, double *jxi_t, int flags,
               void *stream);

/* Section 3.2: the discrete Jacobian of the mesh x (ghost layers valid) from
 * its metrics jxi_x (es_metrics of the same mesh), J = (1/d) sum_k sum_j
 * delta_k[x_j]/dxi_k J dxi_k/dx_j (the cofactor expansion of det dx/dxi along
 * each column k, averaged; delta_k the 2w-order central difference), at
 * interior nodes, ghost layers filled.  Sets J at t = 0 on a mesh that is not
 * uniform (an adapted initial mesh); afterwards J follows eq semi_J.  J is
 * one array of the padded size; it may alias neither x nor jxi_x (ES_EINVAL). */
int es_jacobian(es_ctx *c, const double *x, const double *jxi_x, double *J, void *stream);

/* Sections 3.1-3.4, eq semi_U / eq semi_J with the ES flux eq HOstable (or
 * the EC flux eq ECFlux_curv_2p when dissipation = 0): the semi-discrete
 * right-hand side d(JU)/dt, dJ/dt at interior nodes.  Inputs need valid
 * ghost layers; jxi_t may be NULL (fixed mesh).  dJU/dJ ghost layers are
 * not written; dJU/dJ must not alias the inputs. */
int es_rhs(es_ctx *c, const double *JU, const double *J, const double *jxi_x,
           const double *jxi_t, double *dJU, double *dJ, void *stream);

/* Section 5, SSP-RK3 (Shu-Osher form) stage s = 0, 1, 2 on Q = (JU, J):
 *   Q_out = a_s Q_n + b_s (Q_s + dt L(Q_s)), (a, b) = (0, 1), (3/4, 1/4),
 *   (1/3, 2/3), fused with the right-hand side.  dt is read from dt_dev.
 *   Q_out accumulates the direction sweeps, so it must alias neither Q_s
 *   nor Q_n (ES_EINVAL). */
int es_rk_stage(es_ctx *c, int stage, const double *dt_dev,
                const double *JU_n, const double *J_n,
                const double *JU_s, const double *J_s,
                const double *jxi_x, const double *jxi_t,
                double *JU_out, double *J_out, void *stream);

/* Section 5, eq cfl: lambda = max_i sum_k (|v.n_k| + c |n_k|) / (J_i dxi_k)
 * with n_k = J dxi_k/dx (zero mesh velocity), dt = cfl / lambda; both
 * written to device scalars (either pointer may be NULL). */
int max_wavespeed(es_ctx *c, const double *JU, const double *J,
                  const double *jxi_x, double cfl, double *lambda_dev,
                  double *dt_dev, void *stream);

/* max_wavespeed for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same reduction and result, with no context.  g is validated as by
 * es_create (same error codes) but nothing is allocated: the per-block
 * maxima, lambda, dt and (when status_dev is NULL) the status bits go to a
 * static device array of 2056 doubles (16 KiB) that the library holds on each
 * device it runs on until the process ends.  Any grid es_create accepts
 * fits (at most 2048 partial maxima; ES_EUNSUPPORTED otherwise, and on a
 * device index >= 64).  lambda_dev / dt_dev may be NULL; status_dev, when
 * given, gets ES_ST_NONPHYS or-ed in for a non-physical node.  Calls on one
 * device share that array: calls that overlap on one device (two streams,
 * two host threads) race and must be serialised by the caller. */
int max_wavespeed_noalloc(const es_grid *g, const double *JU, const double *J,
                          const double *jxi_x, double cfl, double *lambda_dev,
                          double *dt_dev, unsigned *status_dev, void *stream);

/* Section 4: monitor eq monitor from sigma = JU/J components, n_smooth
 * passes of the low-pass filter, n_sweeps Jacobi iterations of the mesh
 * equations, movement limiter Delta_tau and disp = Delta_tau (x^[mu] - x_n).
 * Inputs need valid ghost layers; disp gets its ghost layers (component k
 * negated across a non-periodic face of direction k).
 * dtau_dev (1 value) and resid_dev (n_sweeps values: max |x^[nu+1] -
 * x^[nu]|) may be NULL. */
int mesh_redistribute(es_ctx *c, const es_monitor *m, const double *JU,
                      const double *J, const double *x_n, double *disp,
                      double *dtau_dev, double *resid_dev, void *stream);

/* Section 5, total entropy sum_i J_i eta(U_i) dxi_1..dxi_d (fixed-order
 * FP64 sum) into one device scalar. */
int es_entropy(es_ctx *c, const double *JU, const double *J, double *total_dev,
               void *stream);

/* entropy rate sum_i (V_i . dJU_i - phi_i dJ_i) dxi_1..dxi_d (fixed order). */
int es_entropy_rate(es_ctx *c, const double *JU, const double *J,
                    const double *dJU, const double *dJ, double *rate_dev,
                    void *stream);

/* One time step (Sections 4-5): ghost layers, mesh_redistribute when
 * move_mesh, metrics of x_n, dt from max_wavespeed (or dt_fixed > 0), three
 * RK stages on the stage meshes x_n + c_s disp (c = 0, 1, 1/2), and
 * x_{n+1} = x_n + disp.  JU, J, x are updated in place; dt and Delta_tau
 * are written to dt_dev / dtau_dev when given.  m may be NULL when
 * move_mesh = 0.  The context keeps the metrics of x_{n+1} (the c = 1 stage
 * mesh, whose ghost layers the face rules give) with a copy of that mesh,
 * and the next call reuses them when its x_n equals the copy value for value
 * (compared on the device), so x may be changed between calls.  Calls on
 * one context must not overlap. */
int es_step(es_ctx *c, const es_monitor *m, double cfl, double dt_fixed,
            int move_mesh, double *JU, double *J, double *x, double *dt_dev,
            double *dtau_dev, void *stream);

/* Synchronise the stream and return the status word (bits ES_ST_*) in
 * *flags; returns ES_ETANGLE when ES_ST_TANGLE is set (a node with J <= 0
 * also has a non-physical U = JU / J, so the mesh is reported as the
 * cause), else ES_ENONPHYS when ES_ST_NONPHYS is set, else ES_OK.
 * reset != 0 clears the word afterwards. */
int es_status(es_ctx *c, void *stream, unsigned *flags, int reset);

/* Number of padded points P of the context's grid. */
long es_npoints(const es_ctx *c);

/* ------------------------------------------------------------------------
 * Batches: many independent 2D instances of uneven size advanced together,
 * one launch per SSP-RK3 stage.  Each instance is the scheme above on its
 * own periodic grid (its own n, dxi, len); all share nspec, ng, w, the
 * species (gamma, cv, p_inf), chi, weno_eps, dissipation and precision.
 *
 * Per-instance arrays keep the single-instance layouts.  A batched call
 * takes, per argument, a device array of `count` device pointers (entry b
 * for instance b), so a captured graph can be replayed with the same
 * arguments; the tables and the arrays they point to stay caller-owned and
 * must outlive any graph that captured the call.  dt_dev / lambda_dev hold
 * one value per instance.
 * ------------------------------------------------------------------------ */
typedef struct es_batch es_batch;

/* Check the grids (dim must be 2; every field of es_grid that is not an
 * extent, spacing or length must agree with grids[0]) and allocate the
 * batch: work lists of six region shapes (TX x TY nodes on a block: 10 x 10,
 * 15 x 15, 16 x 15, 15 x 16, 18 x 13 and 21 x 21), the wave-speed partials
 * and two stage buffers per instance for es_step_batched.  The shape
 * defaults to 15 x 15 on a persistent grid. */
int es_batch_create(const es_grid *grids, int count, es_batch **out);
int es_batch_destroy(es_batch *b);

typedef struct {
    const double *const *JU_n;   /* Q_n (state at t_n)                         */
    const double *const *J_n;
    const double *const *JU_s;   /* Q_s (stage input), ghost layers filled     */
    const double *const *J_s;
    const double *const *jxi_x;  /* metrics of the (fixed) mesh, ghosts filled */
    const double *const *jxi_t;  /* NULL table: J dxi_k/dt = 0                  */
    double *const *JU_out;       /* Q_{s+1}                                    */
    double *const *J_out;
} es_batch_stage_args;

/* Stage `stage` of Section 5 for every instance (es_rk_stage per instance,
 * with dt_dev[b]).  Writes every interior node of JU_out/J_out and its
 * periodic ghost images, so the output can feed the next stage directly.
 * JU_out/J_out may be the JU_n/J_n arrays (each node's Q_n is read by the
 * thread that then overwrites it) but must not be JU_s/J_s (ES_EINVAL when
 * the tables are the same). */
int es_rk_stage_batched(es_batch *b, int stage, const double *dt_dev,
                        const es_batch_stage_args *a, void *stream);

/* Per-instance CFL wave speed and dt_dev[b] = cfl / lambda_b (eq cfl);
 * lambda_dev may be NULL. */
int max_wavespeed_batched(es_batch *b, const double *const *JU,
                          const double *const *J, const double *const *jxi_x,
                          double cfl, double *lambda_dev, double *dt_dev,
                          void *stream);

/* One fixed-mesh step of every instance: dt_dev[b] from
 * max_wavespeed_batched, then the three stages (buffers owned by the
 * batch); JU, J are advanced in place, ghost layers included.  Four
 * launches plus one wave-speed reduction; nothing synchronises the host, so
 * the call can be captured in a graph. */
int es_step_batched(es_batch *b, double cfl, double *const *JU,
                    double *const *J, const double *const *jxi_x,
                    const double *const *jxi_t, double *dt_dev, void *stream);

/* Autotuner: times stage 0 (output into the batch's own buffers) `reps`
 * times for every region shape with a persistent grid (as many blocks as
 * fit the device at once) and with one block per region, keeps the fastest,
 * and returns it in region_out[0] (TX), region_out[1] (TY) and
 * region_out[2] (1 = persistent).  Synchronises the stream; call it before
 * capturing a graph. */
int es_batch_autotune(es_batch *b, const double *const *JU,
                      const double *const *J, const double *const *jxi_x,
                      const double *const *jxi_t, const double *dt_dev,
                      int reps, void *stream, int *region_out);

/* Select a region shape (one of those of es_batch_create; else ES_EINVAL)
 * and the grid kind by hand. */
int es_batch_set_tiling(es_batch *b, int tx, int ty, int persistent);

/* es_status for the batch's status word. */
int es_batch_status(es_batch *b, void *stream, unsigned *flags, int reset);

#ifdef __cplusplus
}
#endif
#endif
