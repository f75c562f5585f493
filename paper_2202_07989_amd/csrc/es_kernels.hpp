// es_kernels.hpp -- launch interfaces shared by the translation units of libes.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "es_device.hpp"

namespace es {

constexpr int MON_CH = 6;   // monitor channels (variables, or gradient + Laplacian pairs)

struct MonitorP {
    int nsig;
    int sigma[MON_CH];     // 0 rho, 1 rho_1, 2 rho_2, 3 p, 4 |v|, 5 the schlieren function
    double alpha[MON_CH];
    int n_smooth, n_sweeps;
    int form;          // 0: eq monitor; 1: gradient + Laplacian (channels nsig..2 nsig - 1)
    double beta[MON_CH];
    double psi[2];     // Psi = (psi_1 rho_1 + psi_2 rho_2) / rho of the schlieren function
    const double* phi; // the schlieren function with ghost layers (when a variable is 5)
};

struct MeshWork {
    double* grad;   // MON_CH * P
    double* th0;    // P
    double* th1;    // P
    double* xa;     // dim * P
    double* xb;     // dim * P
    double* phi;    // P: the schlieren function
    double* part;   // 8 * 2048 partials
    double* scal;   // 8 scalars: monitor maxima [0..5], Delta_tau [6], max |grad rho| [7]
};

struct RkArgs;

// what a ghost fill treats: plain fields, the mesh x, displacements, the
// metrics J dxi_k/dx_j, the time metrics J dxi_k/dt (they differ only in
// the signs and offsets a mirror across a non-periodic face gives them)
enum { GH_PLAIN = 0, GH_MESH = 1, GH_DISP = 2, GH_JXX = 3, GH_JXT = 4 };

// prescribed conserved states of the inflow faces
struct InflowStates {
    double u[3][2][6];
};

hipError_t fill_ghosts(const Geo& g, double* a, int ncomp, int what, hipStream_t s);
// ghost layers of the state: J, then JU by the reflecting / outflow / inflow
// rules (periodic faces wrap)
hipError_t fill_state(const Geo& g, const InflowStates& in, double* JU, double* J, int nc, int nspec,
                      hipStream_t s);
hipError_t copy(const double* src, double* dst, long n, hipStream_t s);
hipError_t fill_value(double* dst, long n, double v, hipStream_t s);
// *flag = 1 if a and b hold the same n values, else 0 (device-side; NaN never matches)
hipError_t same_values(const double* a, const double* b, long n, int* flag, hipStream_t s);
// dst = src when *flag is 0
hipError_t copy_unless(const double* src, double* dst, long n, const int* flag, hipStream_t s);
hipError_t set_scalar(double* dst, double v, hipStream_t s);
hipError_t jacobian(const Phys& ph, const Geo& g, const double* x, const double* jxx, double* J, hipStream_t s);
// metrics of the stage mesh xn + cs disp, and with jxt the time metrics of the
// mesh velocity disp / dt.  With reuse set on the device, jxx already holds
// the metrics of this mesh (ghost layers included) and only jxt is formed.
hipError_t metrics(const Phys& ph, const Geo& g, const double* xn, const double* disp, double cs,
                   const double* dt_dev, double* jxx, double* jxt, int vcl_only, double* G,
                   hipStream_t s, const int* reuse = nullptr);
hipError_t wavespeed(const Phys& ph, const Geo& g, const double* JU, const double* J, const double* jxx,
                     double cfl, double* part, double* out2, unsigned* status, hipStream_t s);
// number of per-block partials the reductions write for nint interior nodes
int reduction_blocks(long nint);
hipError_t entropy_sum(const Phys& ph, const Geo& g, const double* JU, const double* J, const double* dJU,
                       const double* dJ, double* part, double* out, hipStream_t s);
// with xnext, also x_{n+1} = xn + disp with its ghost layers
hipError_t mesh_redistribute(const Phys& ph, const Geo& g, const MonitorP& mo, const double* JU,
                             const double* J, const double* xn, double* disp, MeshWork& w,
                             double* dtau_out, double* resid_out, unsigned* status, hipStream_t s,
                             double* xnext = nullptr);

struct RkArgs {
    const double* JUn;
    const double* Jn;
    const double* dt;
    double a, b;
    // where the stage result goes; null: over the accumulator.  It may be
    // JUn/Jn themselves (each node's Q_n is read by the thread that then
    // writes the node)
    double* outU = nullptr;
    double* outJ = nullptr;
    // when set, jxt holds -sum_j disp_j J dxi_k/dx_j and the sweeps divide it
    // by this device scalar (the step's dt) as they stage it
    const double* tdiv = nullptr;
};

hipError_t launch_rhs(const Phys& ph, const Geo& g, int mixed, const double* JU, const double* J,
                      const double* jxx, const double* jxt, double* outU, double* outJ,
                      const RkArgs* rk, unsigned* status, hipStream_t s);

// batched 2D instances: device tables of per-instance pointers
struct BatchTables {
    const double* const* JUn;
    const double* const* Jn;
    const double* const* JUs;
    const double* const* Js;
    const double* const* jxx;
    const double* const* jxt;   // may be null (fixed mesh)
    double* const* JUo;
    double* const* Jo;
};

// one region shape of the batched stage: the work list and the grid
struct BatchTiling {
    int v;                // shape index (batch_shape)
    int blocks;           // launch grid (persistent when below ntiles)
    const int4* tiles;    // (instance, x origin, y origin, 0) per region
    int ntiles;
};

// region shapes of the batched stage: v = 0 .. batch_nshapes() - 1 has
// TX x TY nodes on nt threads
int batch_nshapes();
void batch_shape(int v, int* tx, int* ty, int* nt);
hipError_t batch_occupancy(int nspec, int mixed, int recon, int v, int* blocks_per_cu);
hipError_t launch_stage_batched(const Phys& ph, const Geo* geos, int mixed, const BatchTiling& tl,
                                const BatchTables& tb, double ca, double cb, const double* dt_dev,
                                unsigned* status, hipStream_t s);
// per-instance CFL wave speed: wl holds (instance, first row, end row, 0)
// per block, first[b]..first[b+1] the blocks of instance b
hipError_t wavespeed_batched(const Phys& ph, const Geo* geos, const int4* wl, int nwl, const int* first,
                             int count, const double* const* JU, const double* const* J,
                             const double* const* jxx, double cfl, double* part, double* lambda_out,
                             double* dt_out, unsigned* status, hipStream_t s);

}  // namespace es
