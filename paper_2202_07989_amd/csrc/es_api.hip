// es_api.hip -- the C-ABI of libes.so (include/es.h): argument checks,
// per-context workspace, and the native time-step driver.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <limits>
#include <mutex>
#include <vector>

#include "../../include/es.h"
#include "es_kernels.hpp"

using namespace es;

struct es_ctx {
    es_grid grid;
    Phys ph;
    Geo geo;
    InflowStates inflow;
    int device;
    // every buffer below is allocated and initialised by es_create, so no
    // compute call allocates, frees or synchronises the device
    unsigned* status = nullptr;   // device status word
    double* scal = nullptr;       // 16 device scalars: [0] lambda [1] dt [2..] scratch
    double* part = nullptr;       // 4 x 2048 reduction partials
    double* G = nullptr;          // 3D metric pass-1 buffer (9 P)
    MeshWork mesh{};
    double *bufA = nullptr, *bufB = nullptr;
    double *jxx = nullptr, *jxt = nullptr, *disp = nullptr;
    // es_step: the metrics in jxx are those of the mesh mx (ghost layers
    // included; NaN until a step has written it), so the next step reuses
    // them when its x^n equals mx; jxx2 holds the c = 1/2 stage's metrics
    double *mx = nullptr, *jxx2 = nullptr;
    int* reuse = nullptr;         // device flag: jxx holds the metrics of this step's x^n
};

// a batch of independent 2D instances advanced together
struct es_batch {
    int count = 0;
    es_grid grid0{};              // shared physics and scheme (instance 0's grid)
    Phys ph{};
    int device = 0;
    int ncu = 0;
    std::vector<Geo> geo_h;
    Geo* geos = nullptr;          // device copy of geo_h
    unsigned* status = nullptr;
    // work lists of the batched stage, one per region shape (batch_shape)
    static constexpr int NVAR = 6;
    int tx[NVAR] = {}, ty[NVAR] = {};
    int4* tiles[NVAR] = {};
    int ntiles[NVAR] = {};
    int occ[NVAR] = {};           // resident blocks per CU
    int var = 1;                  // chosen shape (15 x 15 until tuned)
    int persistent = 1;           // grid = resident capacity (1) or one block per region (0)
    // wave-speed work list and partials
    int4* wl = nullptr;
    int nwl = 0;
    int* wfirst = nullptr;
    double* part = nullptr;
    // es_step_batched workspace: two stage buffers per instance and their tables
    double* ws = nullptr;
    double** tab = nullptr;       // 4 device tables of count pointers: A_U, A_J, B_U, B_J
};

namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int hip_rc(hipError_t e) { return e == hipSuccess ? ES_OK : ES_EHIP; }

int check_grid(const es_grid* g)
{
    if (!g) return ES_EINVAL;
    if (g->dim != 2 && g->dim != 3) return ES_EUNSUPPORTED;
    if (g->nspec != 1 && g->nspec != 2) return ES_EUNSUPPORTED;
    if (g->w < 1 || g->w > 3 || g->ng < 3) return ES_EUNSUPPORTED;
    if (g->precision != ES_FP64 && g->precision != ES_MIXED) return ES_EUNSUPPORTED;
    if (g->reconstruction != ES_WENO_MR && g->reconstruction != ES_WENO_JS) return ES_EUNSUPPORTED;
    if (g->reconstruction == ES_WENO_JS && g->precision != ES_FP64) return ES_EUNSUPPORTED;
    const int nc = g->nspec + g->dim + 1;
    for (int k = 0; k < g->dim; k++) {
        if (g->n[k] < g->ng || !(g->dxi[k] > 0.0) || !(g->len[k] > 0.0)) return ES_EINVAL;
        for (int s = 0; s < 2; s++)
            if (g->bc[k][s] < ES_BC_PERIODIC || g->bc[k][s] > ES_BC_INFLOW) return ES_EINVAL;
        // a direction is periodic on both faces or on neither
        if ((g->bc[k][0] == ES_BC_PERIODIC) != (g->bc[k][1] == ES_BC_PERIODIC)) return ES_EINVAL;
        if (g->bc[k][0] != ES_BC_PERIODIC && !(g->wall[k][1] > g->wall[k][0])) return ES_EINVAL;
        for (int s = 0; s < 2; s++)
            if (g->bc[k][s] == ES_BC_INFLOW)
                for (int q = 0; q < nc; q++)
                    if (!std::isfinite(g->inflow[k][s][q])) return ES_EINVAL;
    }
    if (g->dim == 2 && g->n[2] != 1) return ES_EINVAL;
    for (int l = 0; l < g->nspec; l++)
        if (!(g->gamma[l] > 1.0) || !(g->cv[l] > 0.0) || !(g->pinf[l] >= 0.0)) return ES_EINVAL;
    if (!(g->chi[0] > 0.0) || !(g->chi[1] > 0.0) || !(g->chi[2] > 0.0) || !(g->weno_eps > 0.0))
        return ES_EINVAL;
    if (!(g->sign_tol >= 0.0 && g->sign_tol < 1.0) || !(g->sign_tol32 >= 0.0 && g->sign_tol32 < 1.0))
        return ES_EINVAL;
    long P = 1;
    for (int k = 0; k < g->dim; k++) P *= (long)(g->n[k] + 2 * g->ng);
    if (P * 9 > (1L << 31) - 1) return ES_EUNSUPPORTED;   // component offsets stay below 2^31
    return ES_OK;
}

void build_params(const es_grid* g, Phys& ph, Geo& geo)
{
    std::memset(&ph, 0, sizeof(ph));
    std::memset(&geo, 0, sizeof(geo));
    ph.nspec = g->nspec;
    ph.dim = g->dim;
    ph.nc = g->nspec + g->dim + 1;
    ph.w = g->w;
    ph.dissipation = g->dissipation ? 1 : 0;
    ph.recon = g->reconstruction;
    for (int l = 0; l < g->nspec; l++) {
        ph.cv[l] = g->cv[l];
        ph.gam[l] = g->gamma[l];
        ph.pinf[l] = g->pinf[l];
        ph.Rg[l] = g->cv[l] * (g->gamma[l] - 1.0);
        ph.cvgam[l] = g->cv[l] * g->gamma[l];
        ph.pinf_tot += g->pinf[l];
    }
    // alpha_{w,m}: sum m alpha = 1, sum m^(2s-1) alpha = 0 (s = 2..w)
    static const double A[3][3] = {{1.0, 0.0, 0.0}, {4.0 / 3.0, -1.0 / 6.0, 0.0},
                                   {3.0 / 2.0, -3.0 / 10.0, 1.0 / 30.0}};
    for (int m = 0; m < 3; m++) ph.alpha[m] = A[g->w - 1][m];
    for (int m = 0; m < 3; m++) ph.chi[m] = g->chi[m];
    ph.eps = g->weno_eps;
    ph.stol64 = g->sign_tol;
    ph.stol32 = g->sign_tol32;
    ph.r21 = g->nspec == 2 ? ph.Rg[1] / ph.Rg[0] : 1.0;
    ph.sr21 = sqrt(ph.r21);
    ph.isr21 = 1.0 / ph.sr21;

    geo.dim = g->dim;
    geo.ng = g->ng;
    for (int k = 0; k < 3; k++) {
        const bool act = k < g->dim;
        geo.n[k] = act ? g->n[k] : 1;
        geo.np[k] = act ? g->n[k] + 2 * g->ng : 1;
        geo.dxi[k] = act ? g->dxi[k] : 1.0;
        geo.idxi[k] = 1.0 / geo.dxi[k];
        geo.len[k] = act ? g->len[k] : 1.0;
        for (int s = 0; s < 2; s++) {
            geo.bc[k][s] = act ? g->bc[k][s] : BC_PERIODIC;
            geo.wall[k][s] = act ? g->wall[k][s] : 0.0;
        }
    }
    geo.P = (long)geo.np[0] * geo.np[1] * geo.np[2];
}

template <typename T>
int dalloc(T** p, size_t count)
{
    if (*p) return ES_OK;
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) == hipSuccess ? ES_OK : ES_EHIP;
}

// the whole workspace of a context, allocated once by es_create and
// initialised there (Theta's ghost layers read as 1 before the first fill,
// and the kept mesh holds NaN, which no mesh equals)
int alloc_workspace(es_ctx* c)
{
    const size_t P = c->geo.P, d = c->geo.dim, nc = c->ph.nc;
    int rc = ES_OK;
    if (c->geo.dim == 3) rc = dalloc(&c->G, 9 * P);
    if (!rc) rc = dalloc(&c->mesh.grad, MON_CH * P);
    if (!rc) rc = dalloc(&c->mesh.th0, P);
    if (!rc) rc = dalloc(&c->mesh.th1, P);
    if (!rc) rc = dalloc(&c->mesh.xa, d * P);
    if (!rc) rc = dalloc(&c->mesh.xb, d * P);
    if (!rc) rc = dalloc(&c->mesh.phi, P);
    if (!rc) rc = dalloc(&c->mesh.part, 8 * 2048);
    if (!rc) rc = dalloc(&c->mesh.scal, 8);
    if (!rc) rc = dalloc(&c->bufA, (nc + 1) * P);
    if (!rc) rc = dalloc(&c->bufB, (nc + 1) * P);
    if (!rc) rc = dalloc(&c->jxx, d * d * P);
    if (!rc) rc = dalloc(&c->jxt, d * P);
    if (!rc) rc = dalloc(&c->disp, d * P);
    if (!rc) rc = dalloc(&c->jxx2, d * d * P);
    if (!rc) rc = dalloc(&c->mx, d * P);
    if (!rc) rc = dalloc(&c->reuse, 1);
    if (rc) return rc;
    if (fill_value(c->mesh.th0, P, 1.0, 0) != hipSuccess) return ES_EHIP;
    if (fill_value(c->mesh.th1, P, 1.0, 0) != hipSuccess) return ES_EHIP;
    if (fill_value(c->mx, d * P, std::numeric_limits<double>::quiet_NaN(), 0) != hipSuccess) return ES_EHIP;
    return hipDeviceSynchronize() == hipSuccess ? ES_OK : ES_EHIP;
}

MonitorP monitor_params(const es_monitor* m)
{
    MonitorP mo{};
    mo.nsig = m->nsig;
    for (int s = 0; s < m->nsig; s++) {
        mo.sigma[s] = m->sigma[s];
        mo.alpha[s] = m->alpha[s];
    }
    mo.n_smooth = m->n_smooth;
    mo.n_sweeps = m->n_sweeps;
    mo.form = m->form;
    for (int s = 0; s < m->nsig; s++) mo.beta[s] = m->form == ES_MONITOR_GRAD_LAP ? m->beta[s] : 0.0;
    mo.psi[0] = m->psi[0];
    mo.psi[1] = m->psi[1];
    mo.phi = nullptr;
    return mo;
}

int check_monitor(const es_monitor* m)
{
    if (!m || m->nsig < 1 || m->nsig > MON_CH || m->n_smooth < 0 || m->n_sweeps < 0 || m->n_sweeps > 4096)
        return ES_EINVAL;
    for (int s = 0; s < m->nsig; s++)
        if (m->sigma[s] < 0 || m->sigma[s] > 5 || !(m->alpha[s] >= 0.0)) return ES_EINVAL;
    if (!std::isfinite(m->psi[0]) || !std::isfinite(m->psi[1])) return ES_EINVAL;
    if (m->form != ES_MONITOR_GRAD2 && m->form != ES_MONITOR_GRAD_LAP) return ES_EINVAL;
    if (m->form == ES_MONITOR_GRAD_LAP) {
        if (m->nsig > 2) return ES_EINVAL;   // gradient and Laplacian maxima share the channels
        for (int s = 0; s < m->nsig; s++)
            if (!(m->beta[s] >= 0.0)) return ES_EINVAL;
    }
    return ES_OK;
}

}  // namespace

extern "C" {

int es_create(const es_grid* g, es_ctx** out)
{
    if (!out) return ES_EINVAL;
    *out = nullptr;
    int rc = check_grid(g);
    if (rc) return rc;
    es_ctx* c = new (std::nothrow) es_ctx();
    if (!c) return ES_EHIP;
    c->grid = *g;
    build_params(g, c->ph, c->geo);
    std::memcpy(c->inflow.u, g->inflow, sizeof(c->inflow.u));
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return ES_EHIP; }
    rc = dalloc(&c->status, 4);
    if (!rc) rc = dalloc(&c->scal, 16);
    if (!rc) rc = dalloc(&c->part, 4 * 2048);
    if (!rc && hipMemset(c->status, 0, 4 * sizeof(unsigned)) != hipSuccess) rc = ES_EHIP;
    if (!rc && hipMemset(c->scal, 0, 16 * sizeof(double)) != hipSuccess) rc = ES_EHIP;
    if (!rc) {
        const double one = 1.0;   // scal[5]: the unit divisor of the step's first metric pass
        if (hipMemcpy(c->scal + 5, &one, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) rc = ES_EHIP;
    }
    if (!rc) rc = alloc_workspace(c);
    if (rc) { es_destroy(c); return rc; }
    *out = c;
    return ES_OK;
}

int es_destroy(es_ctx* c)
{
    if (!c) return ES_EINVAL;
    void* bufs[] = {c->status, c->scal, c->part, c->G, c->mesh.grad, c->mesh.th0, c->mesh.th1,
                    c->mesh.xa, c->mesh.xb, c->mesh.phi, c->mesh.part, c->mesh.scal, c->bufA,
                    c->bufB, c->jxx, c->jxt, c->disp, c->mx, c->jxx2, c->reuse};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    delete c;
    return ES_OK;
}

long es_npoints(const es_ctx* c) { return c ? c->geo.P : 0; }

int es_fill_ghosts(es_ctx* c, double* a, int ncomp, void* stream)
{
    if (!c || !a || ncomp < 1 || ncomp > 16) return ES_EINVAL;
    return hip_rc(fill_ghosts(c->geo, a, ncomp, GH_PLAIN, S(stream)));
}

int es_fill_ghosts_x(es_ctx* c, double* x, void* stream)
{
    if (!c || !x) return ES_EINVAL;
    return hip_rc(fill_ghosts(c->geo, x, c->geo.dim, GH_MESH, S(stream)));
}

int es_fill_ghosts_state(es_ctx* c, double* JU, double* J, void* stream)
{
    if (!c || !JU || !J || JU == J) return ES_EINVAL;
    return hip_rc(fill_state(c->geo, c->inflow, JU, J, c->ph.nc, c->ph.nspec, S(stream)));
}

int es_metrics(es_ctx* c, const double* x_n, const double* disp, double c_s, const double* dt_dev,
               double* jxi_x, double* jxi_t, int flags, void* stream)
{
    if (!c || !jxi_x) return ES_EINVAL;
    const int vcl_only = (flags & ES_METRICS_VCL_ONLY) ? 1 : 0;
    if (!vcl_only && !x_n) return ES_EINVAL;
    if (vcl_only && !jxi_t) return ES_EINVAL;
    if (!std::isfinite(c_s)) return ES_EINVAL;
    return hip_rc(metrics(c->ph, c->geo, x_n, disp, c_s, dt_dev, jxi_x, jxi_t, vcl_only, c->G, S(stream)));
}

int es_jacobian(es_ctx* c, const double* x, const double* jxi_x, double* J, void* stream)
{
    if (!c || !x || !jxi_x || !J) return ES_EINVAL;
    if (J == x || J == jxi_x) return ES_EINVAL;
    return hip_rc(jacobian(c->ph, c->geo, x, jxi_x, J, S(stream)));
}

int es_rhs(es_ctx* c, const double* JU, const double* J, const double* jxi_x, const double* jxi_t,
           double* dJU, double* dJ, void* stream)
{
    if (!c || !JU || !J || !jxi_x || !dJU || !dJ) return ES_EINVAL;
    if (dJU == JU || dJ == J) return ES_EINVAL;
    return hip_rc(launch_rhs(c->ph, c->geo, c->grid.precision == ES_MIXED, JU, J, jxi_x, jxi_t, dJU, dJ,
                             nullptr, c->status, S(stream)));
}

int es_rk_stage(es_ctx* c, int stage, const double* dt_dev, const double* JU_n, const double* J_n,
                const double* JU_s, const double* J_s, const double* jxi_x, const double* jxi_t,
                double* JU_out, double* J_out, void* stream)
{
    if (!c || stage < 0 || stage > 2 || !dt_dev || !JU_n || !J_n || !JU_s || !J_s || !jxi_x || !JU_out ||
        !J_out)
        return ES_EINVAL;
    if (JU_out == JU_s || J_out == J_s || JU_out == JU_n || J_out == J_n) return ES_EINVAL;
    static const double A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    static const double B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    RkArgs rk{JU_n, J_n, dt_dev, A[stage], B[stage]};
    return hip_rc(launch_rhs(c->ph, c->geo, c->grid.precision == ES_MIXED, JU_s, J_s, jxi_x, jxi_t, JU_out,
                             J_out, &rk, c->status, S(stream)));
}

int max_wavespeed(es_ctx* c, const double* JU, const double* J, const double* jxi_x, double cfl,
                  double* lambda_dev, double* dt_dev, void* stream)
{
    if (!c || !JU || !J || !jxi_x || !(cfl > 0.0)) return ES_EINVAL;
    hipStream_t s = S(stream);
    hipError_t e = wavespeed(c->ph, c->geo, JU, J, jxi_x, cfl, c->part, c->scal, c->status, s);
    if (e != hipSuccess) return ES_EHIP;
    if (lambda_dev && copy(c->scal, lambda_dev, 1, s) != hipSuccess) return ES_EHIP;
    if (dt_dev && copy(c->scal + 1, dt_dev, 1, s) != hipSuccess) return ES_EHIP;
    return ES_OK;
}

int mesh_redistribute(es_ctx* c, const es_monitor* m, const double* JU, const double* J, const double* x_n,
                      double* disp, double* dtau_dev, double* resid_dev, void* stream)
{
    if (!c || !JU || !J || !x_n || !disp) return ES_EINVAL;
    const int rc = check_monitor(m);
    if (rc) return rc;
    MonitorP mo = monitor_params(m);
    return hip_rc(es::mesh_redistribute(c->ph, c->geo, mo, JU, J, x_n, disp, c->mesh, dtau_dev, resid_dev,
                                        c->status, S(stream)));
}

int es_entropy(es_ctx* c, const double* JU, const double* J, double* total_dev, void* stream)
{
    if (!c || !JU || !J || !total_dev) return ES_EINVAL;
    return hip_rc(entropy_sum(c->ph, c->geo, JU, J, nullptr, nullptr, c->part, total_dev, S(stream)));
}

int es_entropy_rate(es_ctx* c, const double* JU, const double* J, const double* dJU, const double* dJ,
                    double* rate_dev, void* stream)
{
    if (!c || !JU || !J || !dJU || !dJ || !rate_dev) return ES_EINVAL;
    return hip_rc(entropy_sum(c->ph, c->geo, JU, J, dJU, dJ, c->part, rate_dev, S(stream)));
}

int es_step(es_ctx* c, const es_monitor* m, double cfl, double dt_fixed, int move_mesh, double* JU,
            double* J, double* x, double* dt_dev, double* dtau_dev, void* stream)
{
    if (!c || !JU || !J || !x) return ES_EINVAL;
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return ES_EINVAL;
    if (move_mesh) {
        const int rc = check_monitor(m);
        if (rc) return rc;
    }
    hipStream_t s = S(stream);
    const Geo& g = c->geo;
    const Phys& ph = c->ph;
    const long P = g.P;
    const int nc = ph.nc, d = g.dim;
    const int mixed = c->grid.precision == ES_MIXED;
    double* dt = c->scal + 1;
    double* dtau = c->scal + 2;
#define ES_TRY(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return ES_EHIP;     \
    } while (0)

    ES_TRY(fill_state(g, c->inflow, JU, J, nc, ph.nspec, s));
    ES_TRY(fill_ghosts(g, x, d, GH_MESH, s));
    // x^n is as a rule the previous step's c = 1 stage mesh, whose metrics
    // that step left in jxx beside a copy mx of the mesh: a device-side
    // comparison of x^n with mx (before the mesh step below overwrites mx)
    // decides whether they are reused or formed afresh, so a caller may
    // change x between steps
    ES_TRY(same_values(x, c->mx, d * P, c->reuse, s));
    const double* disp = nullptr;
    if (move_mesh) {
        // the displacement, and in mx the c = 1 stage mesh x^{n+1} = x^n + disp
        // with its ghost layers by the face rules
        MonitorP mo = monitor_params(m);
        ES_TRY(es::mesh_redistribute(ph, g, mo, JU, J, x, c->disp, c->mesh, dtau, nullptr, c->status, s,
                                     c->mx));
        disp = c->disp;
    } else {
        ES_TRY(set_scalar(dtau, 0.0, s));
    }
    // metrics of x^n and the CFL step (zero mesh velocity).  With a moving
    // mesh the same pass leaves -sum_j disp_j J dxi_k/dx_j in jxt (divided by
    // the device scalar 1); stage 0's sweeps divide it by dt once dt exists
    ES_TRY(metrics(ph, g, x, disp, 0.0, disp ? c->scal + 5 : nullptr, c->jxx, disp ? c->jxt : nullptr, 0,
                   c->G, s, c->reuse));
    // a fixed mesh keeps these metrics for the steps that follow
    if (!disp) ES_TRY(copy_unless(x, c->mx, d * P, c->reuse, s));
    if (dt_fixed > 0.0) ES_TRY(set_scalar(dt, dt_fixed, s));
    else ES_TRY(wavespeed(ph, g, JU, J, c->jxx, cfl, c->part, c->scal, c->status, s));
    static const double A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    static const double B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    static const double Cs[3] = {0.0, 1.0, 0.5};
    // Q_n is the caller's (JU, J) itself: stages 0 and 1 only read it, and
    // stage 2 accumulates its direction sweeps in bufA (free by then) and
    // writes Q_{n+1} over Q_n, each node by the thread that read its Q_n
    const double* inU = JU;
    const double* inJ = J;
    double* accs[3][2] = {{c->bufA, c->bufA + nc * P}, {c->bufB, c->bufB + nc * P}, {c->bufA, c->bufA + nc * P}};
    double* outs[3][2] = {{c->bufA, c->bufA + nc * P}, {c->bufB, c->bufB + nc * P}, {JU, J}};
    double* jxs[3] = {c->jxx, c->jxx, disp ? c->jxx2 : c->jxx};
    for (int st = 0; st < 3; st++) {
        // stage mesh x^n + c_s disp (stage 0 has it from the pass above).
        // The c = 1 stage mesh is x^{n+1}, formed once in mx by the mesh step;
        // its metrics stay in jxx for the next step, and the c = 1/2 stage's
        // go to jxx2
        if (disp && st == 1) {
            ES_TRY(metrics(ph, g, c->mx, disp, 0.0, dt, c->jxx, c->jxt, 0, c->G, s));
        } else if (disp && st == 2) {
            ES_TRY(metrics(ph, g, x, disp, Cs[st], dt, c->jxx2, c->jxt, 0, c->G, s));
        }
        RkArgs rk{JU, J, dt, A[st], B[st], outs[st][0], outs[st][1], (disp && st == 0) ? dt : nullptr};
        ES_TRY(launch_rhs(ph, g, mixed, inU, inJ, jxs[st], disp ? c->jxt : nullptr, accs[st][0], accs[st][1],
                          &rk, c->status, s));
        ES_TRY(fill_state(g, c->inflow, outs[st][0], outs[st][1], nc, ph.nspec, s));
        inU = outs[st][0];
        inJ = outs[st][1];
    }
    // x^{n+1} with its ghost layers
    if (disp) ES_TRY(copy(c->mx, x, d * P, s));
    if (dt_dev) ES_TRY(copy(dt, dt_dev, 1, s));
    if (dtau_dev) ES_TRY(copy(dtau, dtau_dev, 1, s));
#undef ES_TRY
    return ES_OK;
}

int es_status(es_ctx* c, void* stream, unsigned* flags, int reset)
{
    if (!c) return ES_EINVAL;
    hipStream_t s = S(stream);
    unsigned h = 0;
    if (hipMemcpyAsync(&h, c->status, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess) return ES_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return ES_EHIP;
    if (reset) {
        if (hipMemsetAsync(c->status, 0, sizeof(unsigned), s) != hipSuccess) return ES_EHIP;
        if (hipStreamSynchronize(s) != hipSuccess) return ES_EHIP;
    }
    if (flags) *flags = h;
    if (h & ES_ST_TANGLE) return ES_ETANGLE;
    if (h & ES_ST_NONPHYS) return ES_ENONPHYS;
    return ES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched 2D instances
// ---------------------------------------------------------------------------
namespace {

bool same_scheme(const es_grid& a, const es_grid& b)
{
    if (a.dim != b.dim || a.nspec != b.nspec || a.ng != b.ng || a.w != b.w || a.precision != b.precision ||
        a.dissipation != b.dissipation || a.weno_eps != b.weno_eps || a.reconstruction != b.reconstruction ||
        a.sign_tol != b.sign_tol || a.sign_tol32 != b.sign_tol32)
        return false;
    for (int l = 0; l < a.nspec; l++)
        if (a.gamma[l] != b.gamma[l] || a.cv[l] != b.cv[l] || a.pinf[l] != b.pinf[l]) return false;
    for (int m = 0; m < 3; m++)
        if (a.chi[m] != b.chi[m]) return false;
    return true;
}

BatchTiling batch_tiling(const es_batch* b)
{
    BatchTiling tl{};
    tl.v = b->var;
    tl.tiles = b->tiles[b->var];
    tl.ntiles = b->ntiles[b->var];
    const long cap = (long)b->occ[b->var] * b->ncu;
    tl.blocks = (b->persistent && cap > 0 && cap < tl.ntiles) ? (int)cap : tl.ntiles;
    return tl;
}

int batch_stage(es_batch* b, int stage, const double* dt_dev, const BatchTables& tb, hipStream_t s)
{
    static const double A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    static const double B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    return hip_rc(launch_stage_batched(b->ph, b->geos, b->grid0.precision == ES_MIXED, batch_tiling(b), tb,
                                       A[stage], B[stage], dt_dev, b->status, s));
}

}  // namespace

extern "C" {

int es_batch_create(const es_grid* grids, int count, es_batch** out)
{
    if (!out) return ES_EINVAL;
    *out = nullptr;
    if (!grids || count < 1) return ES_EINVAL;
    for (int i = 0; i < count; i++) {
        const int rc = check_grid(&grids[i]);
        if (rc) return rc;
        if (grids[i].dim != 2) return ES_EUNSUPPORTED;
        for (int k = 0; k < 2; k++)
            if (grids[i].bc[k][0] != ES_BC_PERIODIC) return ES_EUNSUPPORTED;   // batches are periodic
        if (!same_scheme(grids[0], grids[i])) return ES_EINVAL;
    }
    es_batch* b = new (std::nothrow) es_batch();
    if (!b) return ES_EHIP;
    b->count = count;
    b->grid0 = grids[0];
    Geo g0;
    build_params(&grids[0], b->ph, g0);
    b->geo_h.resize(count);
    size_t ws_doubles = 0;
    const int nc = b->ph.nc;
    for (int i = 0; i < count; i++) {
        Phys ph;
        build_params(&grids[i], ph, b->geo_h[i]);
        ws_doubles += 2 * (size_t)(nc + 1) * b->geo_h[i].P;
    }
    int rc = ES_OK;
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
        rc = ES_EHIP;
    if (!rc) rc = dalloc(&b->geos, count);
    if (!rc) rc = dalloc(&b->status, 4);
    if (!rc && hipMemcpy(b->geos, b->geo_h.data(), count * sizeof(Geo), hipMemcpyHostToDevice) != hipSuccess)
        rc = ES_EHIP;
    if (!rc && hipMemset(b->status, 0, 4 * sizeof(unsigned)) != hipSuccess) rc = ES_EHIP;
    // region work lists
    if (batch_nshapes() != es_batch::NVAR) rc = ES_EHIP;
    for (int v = 0; v < es_batch::NVAR && !rc; v++) {
        int nt = 0;
        batch_shape(v, &b->tx[v], &b->ty[v], &nt);
        std::vector<int4> tl;
        for (int i = 0; i < count; i++)
            for (int oy = 0; oy < b->geo_h[i].n[1]; oy += b->ty[v])
                for (int ox = 0; ox < b->geo_h[i].n[0]; ox += b->tx[v]) tl.push_back(make_int4(i, ox, oy, 0));
        b->ntiles[v] = (int)tl.size();
        rc = dalloc(&b->tiles[v], tl.size());
        if (!rc && hipMemcpy(b->tiles[v], tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess)
            rc = ES_EHIP;
        if (!rc && batch_occupancy(b->ph.nspec, b->grid0.precision == ES_MIXED, b->ph.recon, v, &b->occ[v]) != hipSuccess)
            rc = ES_EHIP;
    }
    // wave-speed work list: blocks of about 4096 nodes
    if (!rc) {
        std::vector<int4> wl;
        std::vector<int> first(count + 1, 0);
        for (int i = 0; i < count; i++) {
            const int n0 = b->geo_h[i].n[0], n1 = b->geo_h[i].n[1];
            const int rows = std::max(1, 4096 / n0);
            first[i] = (int)wl.size();
            for (int j = 0; j < n1; j += rows) wl.push_back(make_int4(i, j, std::min(n1, j + rows), 0));
        }
        first[count] = (int)wl.size();
        b->nwl = (int)wl.size();
        rc = dalloc(&b->wl, wl.size());
        if (!rc) rc = dalloc(&b->wfirst, first.size());
        if (!rc) rc = dalloc(&b->part, wl.size());
        if (!rc && (hipMemcpy(b->wl, wl.data(), wl.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(b->wfirst, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice) !=
                        hipSuccess))
            rc = ES_EHIP;
    }
    // step workspace and its pointer tables
    if (!rc) rc = dalloc(&b->ws, ws_doubles);
    if (!rc) rc = dalloc(&b->tab, 4 * (size_t)count);
    if (!rc) {
        std::vector<double*> t(4 * (size_t)count);
        double* p = b->ws;
        for (int i = 0; i < count; i++) {
            const size_t P = b->geo_h[i].P;
            t[0 * count + i] = p;
            t[1 * count + i] = p + nc * P;
            p += (nc + 1) * P;
            t[2 * count + i] = p;
            t[3 * count + i] = p + nc * P;
            p += (nc + 1) * P;
        }
        if (hipMemcpy(b->tab, t.data(), t.size() * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess)
            rc = ES_EHIP;
    }
    if (rc) {
        es_batch_destroy(b);
        return rc;
    }
    *out = b;
    return ES_OK;
}

int es_batch_destroy(es_batch* b)
{
    if (!b) return ES_EINVAL;
    void* bufs[] = {b->geos, b->status, b->wl, b->wfirst, b->part, b->ws, b->tab};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    for (int v = 0; v < es_batch::NVAR; v++)
        if (b->tiles[v]) (void)hipFree(b->tiles[v]);
    delete b;
    return ES_OK;
}

int max_wavespeed_batched(es_batch* b, const double* const* JU, const double* const* J,
                          const double* const* jxi_x, double cfl, double* lambda_dev, double* dt_dev,
                          void* stream)
{
    if (!b || !JU || !J || !jxi_x || !dt_dev || !(cfl > 0.0)) return ES_EINVAL;
    return hip_rc(wavespeed_batched(b->ph, b->geos, b->wl, b->nwl, b->wfirst, b->count, JU, J, jxi_x, cfl,
                                    b->part, lambda_dev, dt_dev, b->status, S(stream)));
}

int es_rk_stage_batched(es_batch* b, int stage, const double* dt_dev, const es_batch_stage_args* a,
                        void* stream)
{
    if (!b || !a || stage < 0 || stage > 2 || !dt_dev || !a->JU_n || !a->J_n || !a->JU_s || !a->J_s ||
        !a->jxi_x || !a->JU_out || !a->J_out)
        return ES_EINVAL;
    if ((const void*)a->JU_out == (const void*)a->JU_s || (const void*)a->J_out == (const void*)a->J_s)
        return ES_EINVAL;
    BatchTables tb{a->JU_n, a->J_n, a->JU_s, a->J_s, a->jxi_x, a->jxi_t, a->JU_out, a->J_out};
    return batch_stage(b, stage, dt_dev, tb, S(stream));
}

int es_step_batched(es_batch* b, double cfl, double* const* JU, double* const* J,
                    const double* const* jxi_x, const double* const* jxi_t, double* dt_dev, void* stream)
{
    if (!b || !JU || !J || !jxi_x || !dt_dev || !(cfl > 0.0)) return ES_EINVAL;
    hipStream_t s = S(stream);
    const int n = b->count;
    const double* const* cU = JU;
    const double* const* cJ = J;
    double* const* AU = b->tab;
    double* const* AJ = b->tab + n;
    double* const* BU = b->tab + 2 * n;
    double* const* BJ = b->tab + 3 * n;
    int rc = max_wavespeed_batched(b, cU, cJ, jxi_x, cfl, nullptr, dt_dev, stream);
    if (rc) return rc;
    // Q1 = Qn + dt L(Qn); Q2 = 3/4 Qn + 1/4 (Q1 + dt L(Q1)); Qn+1 = 1/3 Qn + 2/3 (Q2 + dt L(Q2)),
    // the last written over Qn (each node's Qn is read by the thread that overwrites it)
    rc = batch_stage(b, 0, dt_dev, BatchTables{cU, cJ, cU, cJ, jxi_x, jxi_t, AU, AJ}, s);
    if (!rc) rc = batch_stage(b, 1, dt_dev, BatchTables{cU, cJ, AU, AJ, jxi_x, jxi_t, BU, BJ}, s);
    if (!rc) rc = batch_stage(b, 2, dt_dev, BatchTables{cU, cJ, BU, BJ, jxi_x, jxi_t, JU, J}, s);
    return rc;
}

int es_batch_autotune(es_batch* b, const double* const* JU, const double* const* J,
                      const double* const* jxi_x, const double* const* jxi_t, const double* dt_dev,
                      int reps, void* stream, int* region_out)
{
    if (!b || !JU || !J || !jxi_x || !dt_dev || reps < 1) return ES_EINVAL;
    hipStream_t s = S(stream);
    const int n = b->count;
    BatchTables tb{JU, J, JU, J, jxi_x, jxi_t, b->tab, b->tab + n};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return ES_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return ES_EHIP; }
    float best = 1e30f;
    int best_var = b->var, best_pers = b->persistent;
    int rc = ES_OK;
    for (int v = 0; v < es_batch::NVAR && !rc; v++) {
        for (int pers = 0; pers < 2 && !rc; pers++) {
            b->var = v;
            b->persistent = pers;
            rc = batch_stage(b, 0, dt_dev, tb, s);                   // warm-up
            if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = ES_EHIP;
            for (int r = 0; r < reps && !rc; r++) rc = batch_stage(b, 0, dt_dev, tb, s);
            if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = ES_EHIP;
            if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = ES_EHIP;
            float ms = 0.0f;
            if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = ES_EHIP;
            if (!rc && ms < best) {
                best = ms;
                best_var = v;
                best_pers = pers;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->var = best_var;
    b->persistent = best_pers;
    if (region_out) {
        region_out[0] = b->tx[best_var];
        region_out[1] = b->ty[best_var];
        region_out[2] = best_pers;
    }
    return rc;
}

int es_batch_set_tiling(es_batch* b, int tx, int ty, int persistent)
{
    if (!b) return ES_EINVAL;
    for (int v = 0; v < es_batch::NVAR; v++)
        if (b->tx[v] == tx && b->ty[v] == ty) {
            b->var = v;
            b->persistent = persistent ? 1 : 0;
            return ES_OK;
        }
    return ES_EINVAL;
}

int es_batch_status(es_batch* b, void* stream, unsigned* flags, int reset)
{
    if (!b) return ES_EINVAL;
    hipStream_t s = S(stream);
    unsigned h = 0;
    if (hipMemcpyAsync(&h, b->status, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess) return ES_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return ES_EHIP;
    if (reset) {
        if (hipMemsetAsync(b->status, 0, sizeof(unsigned), s) != hipSuccess) return ES_EHIP;
        if (hipStreamSynchronize(s) != hipSuccess) return ES_EHIP;
    }
    if (flags) *flags = h;
    if (h & ES_ST_TANGLE) return ES_ETANGLE;
    if (h & ES_ST_NONPHYS) return ES_ENONPHYS;
    return ES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// max_wavespeed_noalloc: the CFL reduction for callers that cannot allocate.
// Its scratch (per-block maxima, lambda and dt, a status word) is a static
// device array; host code reaches it only through the address that
// hipGetSymbolAddress returns on each device (the array's name is a host-side
// stand-in, not a device address).
// ---------------------------------------------------------------------------
namespace {
constexpr int NOALLOC_PARTS = 2048;                  // per-block maxima
constexpr int NOALLOC_DOUBLES = NOALLOC_PARTS + 8;   // + lambda, dt, status word
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
std::mutex scratch_mu;
double* scratch_dev[NOALLOC_MAX_DEVICES] = {};

// device address of scratch on device dev (current), looked up once per device
int scratch_address(int dev, double** out)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ES_EHIP;
        scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = scratch_dev[dev];
    return ES_OK;
}
}  // namespace

extern "C" int max_wavespeed_noalloc(const es_grid* g, const double* JU, const double* J, const double* jxi_x,
                                     double cfl, double* lambda_dev, double* dt_dev, unsigned* status_dev,
                                     void* stream)
{
    if (!JU || !J || !jxi_x || !(cfl > 0.0)) return ES_EINVAL;
    int rc = check_grid(g);
    if (rc) return rc;
    Phys ph;
    Geo geo;
    build_params(g, ph, geo);
    const long nint = (long)geo.n[0] * geo.n[1] * geo.n[2];
    if (reduction_blocks(nint) > NOALLOC_PARTS) return ES_EUNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ES_EHIP;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return ES_EUNSUPPORTED;
    double* sc = nullptr;
    rc = scratch_address(dev, &sc);
    if (rc) return rc;
    // every partial the finishing pass reads is written by its block first,
    // and the status word in the scratch is only ever or-ed (never read), so
    // nothing has to be cleared between calls
    unsigned* st = status_dev ? status_dev : reinterpret_cast<unsigned*>(sc + NOALLOC_PARTS + 2);
    hipStream_t s = S(stream);
    if (wavespeed(ph, geo, JU, J, jxi_x, cfl, sc, sc + NOALLOC_PARTS, st, s) != hipSuccess) return ES_EHIP;
    if (lambda_dev && copy(sc + NOALLOC_PARTS, lambda_dev, 1, s) != hipSuccess) return ES_EHIP;
    if (dt_dev && copy(sc + NOALLOC_PARTS + 1, dt_dev, 1, s) != hipSuccess) return ES_EHIP;
    return ES_OK;
}
