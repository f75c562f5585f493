// es_api.hip -- the C-ABI of libes.so (include/es.h): argument checks,
// per-context workspace, and the native time-step driver.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "../../include/es.h"
#include "es_kernels.hpp"

using namespace es;

struct es_ctx {
    es_grid grid;
    Phys ph;
    Geo geo;
    int device;
    unsigned* status = nullptr;   // device status word
    double* scal = nullptr;       // 16 device scalars: [0] lambda [1] dt [2..] scratch
    double* part = nullptr;       // 4 x 2048 reduction partials
    // lazily sized workspace
    double* G = nullptr;          // 3D metric pass-1 buffer (9 P)
    MeshWork mesh{};
    bool mesh_ready = false;
    int mesh_nsig = 0;
    double *JUn = nullptr, *Jn = nullptr, *bufA = nullptr, *bufB = nullptr;
    double *jxx = nullptr, *jxt = nullptr, *disp = nullptr;
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
    for (int k = 0; k < g->dim; k++)
        if (g->n[k] < g->ng || !(g->dxi[k] > 0.0) || !(g->len[k] > 0.0)) return ES_EINVAL;
    if (g->dim == 2 && g->n[2] != 1) return ES_EINVAL;
    for (int l = 0; l < g->nspec; l++)
        if (!(g->gamma[l] > 1.0) || !(g->cv[l] > 0.0) || !(g->pinf[l] >= 0.0)) return ES_EINVAL;
    if (!(g->chi[0] > 0.0) || !(g->chi[1] > 0.0) || !(g->chi[2] > 0.0) || !(g->weno_eps > 0.0))
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
    ph.ichi3 = 1.0 / g->chi[2];
    ph.c1c3 = g->chi[0] / g->chi[2];
    ph.c2c3 = g->chi[1] / g->chi[2];
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
    }
    geo.P = (long)geo.np[0] * geo.np[1] * geo.np[2];
}

template <typename T>
int dalloc(T** p, size_t count)
{
    if (*p) return ES_OK;
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) == hipSuccess ? ES_OK : ES_EHIP;
}

int ensure_metric_ws(es_ctx* c)
{
    if (c->geo.dim == 3) return dalloc(&c->G, 9 * (size_t)c->geo.P);
    return ES_OK;
}

int ensure_mesh_ws(es_ctx* c, int nsig)
{
    const size_t P = c->geo.P, d = c->geo.dim;
    if (c->mesh_ready && nsig <= c->mesh_nsig) return ES_OK;
    int rc = dalloc(&c->mesh.grad, 4 * P);
    if (!rc) rc = dalloc(&c->mesh.th0, P);
    if (!rc) rc = dalloc(&c->mesh.th1, P);
    if (!rc) rc = dalloc(&c->mesh.xa, d * P);
    if (!rc) rc = dalloc(&c->mesh.xb, d * P);
    if (!rc) rc = dalloc(&c->mesh.part, 4 * 2048);
    if (!rc) rc = dalloc(&c->mesh.scal, 8);
    if (rc) return rc;
    // theta ghosts are read by the filter before the first fill
    if (fill_value(c->mesh.th0, P, 1.0, 0) != hipSuccess) return ES_EHIP;
    if (fill_value(c->mesh.th1, P, 1.0, 0) != hipSuccess) return ES_EHIP;
    c->mesh_ready = true;
    c->mesh_nsig = 4;
    return hipDeviceSynchronize() == hipSuccess ? ES_OK : ES_EHIP;
}

int ensure_step_ws(es_ctx* c)
{
    const size_t P = c->geo.P, d = c->geo.dim, nc = c->ph.nc;
    int rc = dalloc(&c->JUn, nc * P);
    if (!rc) rc = dalloc(&c->Jn, P);
    if (!rc) rc = dalloc(&c->bufA, (nc + 1) * P);
    if (!rc) rc = dalloc(&c->bufB, (nc + 1) * P);
    if (!rc) rc = dalloc(&c->jxx, d * d * P);
    if (!rc) rc = dalloc(&c->jxt, d * P);
    if (!rc) rc = dalloc(&c->disp, d * P);
    if (!rc) rc = ensure_metric_ws(c);
    return rc;
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
    return mo;
}

int check_monitor(const es_monitor* m)
{
    if (!m || m->nsig < 1 || m->nsig > 4 || m->n_smooth < 0 || m->n_sweeps < 0 || m->n_sweeps > 4096)
        return ES_EINVAL;
    for (int s = 0; s < m->nsig; s++)
        if (m->sigma[s] < 0 || m->sigma[s] > 3 || !(m->alpha[s] >= 0.0)) return ES_EINVAL;
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
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return ES_EHIP; }
    rc = dalloc(&c->status, 4);
    if (!rc) rc = dalloc(&c->scal, 16);
    if (!rc) rc = dalloc(&c->part, 4 * 2048);
    if (!rc && hipMemset(c->status, 0, 4 * sizeof(unsigned)) != hipSuccess) rc = ES_EHIP;
    if (!rc && hipMemset(c->scal, 0, 16 * sizeof(double)) != hipSuccess) rc = ES_EHIP;
    if (rc) { es_destroy(c); return rc; }
    *out = c;
    return ES_OK;
}

int es_destroy(es_ctx* c)
{
    if (!c) return ES_EINVAL;
    void* bufs[] = {c->status, c->scal, c->part, c->G, c->mesh.grad, c->mesh.th0, c->mesh.th1,
                    c->mesh.xa, c->mesh.xb, c->mesh.part, c->mesh.scal, c->JUn, c->Jn, c->bufA,
                    c->bufB, c->jxx, c->jxt, c->disp};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    delete c;
    return ES_OK;
}

long es_npoints(const es_ctx* c) { return c ? c->geo.P : 0; }

int es_fill_ghosts(es_ctx* c, double* a, int ncomp, void* stream)
{
    if (!c || !a || ncomp < 1 || ncomp > 16) return ES_EINVAL;
    return hip_rc(fill_ghosts(c->geo, a, ncomp, 0, S(stream)));
}

int es_fill_ghosts_x(es_ctx* c, double* x, void* stream)
{
    if (!c || !x) return ES_EINVAL;
    return hip_rc(fill_ghosts(c->geo, x, c->geo.dim, 1, S(stream)));
}

int es_metrics(es_ctx* c, const double* x_n, const double* disp, double c_s, const double* dt_dev,
               double* jxi_x, double* jxi_t, int flags, void* stream)
{
    if (!c || !jxi_x) return ES_EINVAL;
    const int vcl_only = (flags & ES_METRICS_VCL_ONLY) ? 1 : 0;
    if (!vcl_only && !x_n) return ES_EINVAL;
    if (vcl_only && !jxi_t) return ES_EINVAL;
    if (!std::isfinite(c_s)) return ES_EINVAL;
    if (!vcl_only) {
        int rc = ensure_metric_ws(c);
        if (rc) return rc;
    }
    return hip_rc(metrics(c->ph, c->geo, x_n, disp, c_s, dt_dev, jxi_x, jxi_t, vcl_only, c->G, S(stream)));
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
    int rc = check_monitor(m);
    if (rc) return rc;
    rc = ensure_mesh_ws(c, m->nsig);
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
        int rc = check_monitor(m);
        if (rc) return rc;
        rc = ensure_mesh_ws(c, m->nsig);
        if (rc) return rc;
    }
    int rc = ensure_step_ws(c);
    if (rc) return rc;
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

    ES_TRY(fill_ghosts(g, JU, nc, 0, s));
    ES_TRY(fill_ghosts(g, J, 1, 0, s));
    ES_TRY(fill_ghosts(g, x, d, 1, s));
    const double* disp = nullptr;
    if (move_mesh) {
        MonitorP mo = monitor_params(m);
        ES_TRY(es::mesh_redistribute(ph, g, mo, JU, J, x, c->disp, c->mesh, dtau, nullptr, c->status, s));
        disp = c->disp;
    } else {
        ES_TRY(set_scalar(dtau, 0.0, s));
    }
    // metrics of x^n and the CFL step (zero mesh velocity)
    ES_TRY(metrics(ph, g, x, nullptr, 0.0, nullptr, c->jxx, nullptr, 0, c->G, s));
    if (dt_fixed > 0.0) ES_TRY(set_scalar(dt, dt_fixed, s));
    else ES_TRY(wavespeed(ph, g, JU, J, c->jxx, cfl, c->part, c->scal, c->status, s));
    ES_TRY(copy(JU, c->JUn, nc * P, s));
    ES_TRY(copy(J, c->Jn, P, s));
    static const double A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    static const double B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    static const double Cs[3] = {0.0, 1.0, 0.5};
    const double* inU = JU;
    const double* inJ = J;
    double* outs[3][2] = {{c->bufA, c->bufA + nc * P}, {c->bufB, c->bufB + nc * P}, {JU, J}};
    for (int st = 0; st < 3; st++) {
        // stage mesh x^n + c_s disp: stage 0 keeps the spatial metrics of x^n
        if (disp) ES_TRY(metrics(ph, g, x, disp, Cs[st], dt, c->jxx, c->jxt, st == 0 ? 1 : 0, c->G, s));
        RkArgs rk{c->JUn, c->Jn, dt, A[st], B[st]};
        ES_TRY(launch_rhs(ph, g, mixed, inU, inJ, c->jxx, disp ? c->jxt : nullptr, outs[st][0], outs[st][1],
                          &rk, c->status, s));
        ES_TRY(fill_ghosts(g, outs[st][0], nc, 0, s));
        ES_TRY(fill_ghosts(g, outs[st][1], 1, 0, s));
        inU = outs[st][0];
        inJ = outs[st][1];
    }
    if (disp) ES_TRY(add_inplace(x, disp, d * P, s));
    ES_TRY(fill_ghosts(g, x, d, 1, s));
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
    if (h & ES_ST_NONPHYS) return ES_ENONPHYS;
    if (h & ES_ST_TANGLE) return ES_ETANGLE;
    return ES_OK;
}

}  // extern "C"
