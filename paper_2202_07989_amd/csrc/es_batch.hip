// es_batch.hip -- one SSP-RK3 stage (Section 5) of many independent 2D
// instances of uneven size in one persistent launch; each instance is the
// semi-discrete scheme of Sections 3.1-3.4 on its own periodic grid.
//
// The work list holds regions of TX x TY nodes of every instance (the
// autotuner picks the shape).  A block takes regions round-robin and, for each,
//   - stages the node quantities of the region plus a 3-node halo along both
//     directions (a plus-shaped patch) in LDS once,
//   - sweeps direction 1 and then direction 2 over the patch with the
//     interface-flux scheme of interface_fluxes() (the metrics of the sweep
//     direction are reloaded between the sweeps), keeping each node's
//     right-hand side in registers across the two sweeps,
//   - writes the Shu-Osher combination to the node and to its periodic ghost
//     images, so the next stage reads complete ghost layers with no fill.
// A region's right-hand side depends only on its patch, so regions need no
// ordering and the launch has no grid-wide synchronisation.
#include "es_flux.hpp"

namespace es {

template <int N, int TX, int TY, int NT, typename R, int RC>
__global__ void __launch_bounds__(NT)
k_stage2d_batched(Phys ph, const Geo* __restrict__ geos, const int4* __restrict__ tiles, int ntiles,
                  BatchTables tb, double ca, double cb, const double* __restrict__ dt_dev,
                  unsigned* __restrict__ status)
{
    constexpr int D = 2;
    constexpr int NC = N + D + 1;
    constexpr int NEX = TX + 6, NEY = TY + 6;   // patch: region + 3-node halo on each side
    constexpr int NN = NEX * NEY;
    // per sweep: TX + 1 interfaces on TY lines (x), TY + 1 on TX lines (y);
    // exchange slots: along + 4 per line
    constexpr int NX = ((TX + 4) * TY > (TY + 4) * TX) ? (TX + 4) * TY : (TY + 4) * TX;
    constexpr int NW = NT / 64;
    static_assert((TX + 1) * TY <= NT && (TY + 1) * TX <= NT && 3 * TX <= 64 && 3 * TY <= 64 && NT % 64 == 0,
                  "region does not fit");
    __shared__ NodeTile<N, D, NN> S;
    __shared__ R Xbuf[NC * NX];

    const int t = threadIdx.x;
    auto lidx = [](int lx, int ly) { return lx + NEX * ly; };
    unsigned bad = 0;

    for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
        const int4 tw = tiles[w];
        const int bi = tw.x, ox = tw.y, oy = tw.z;
        const Geo g = geos[bi];
        const long P = g.P;
        const int nx = g.n[0], ny = g.n[1], np0 = g.np[0], ng = g.ng;
        const double* __restrict__ JUs = tb.JUs[bi];
        const double* __restrict__ Js = tb.Js[bi];
        const double* __restrict__ jxx = tb.jxx[bi];
        const double* __restrict__ jxt = tb.jxt ? tb.jxt[bi] : nullptr;
        // interior coordinates (gx, gy) in [-ng, n + ng) -> padded index
        auto gidx = [&](int gx, int gy) -> long { return (long)(gy + ng) * np0 + (gx + ng); };

        // ---- node quantities of the plus-shaped patch ---------------------
        for (int q = t; q < NN; q += NT) {
            const int lx = q % NEX, ly = q / NEX;
            const bool cx = lx >= 3 && lx < 3 + TX, cy = ly >= 3 && ly < 3 + TY;
            if (!(cx || cy)) continue;                       // corners are never read
            const int gx = ox + lx - 3, gy = oy + ly - 3;
            if (gx >= nx + 3 || gy >= ny + 3) continue;      // beyond a ragged last region
            bad |= node_state<N, D, NN>(ph, S, q, JUs, Js, P, gidx(gx, gy));
        }

        // node owned by this thread in the node phases
        const int ni = t % TX, nj = t / TX;
        double acc[NC], accJ = 0.0;
#pragma unroll
        for (int cc = 0; cc < NC; cc++) acc[cc] = 0.0;

        auto sweep = [&](auto kc) {
            constexpr int K = decltype(kc)::value;
            constexpr int TL = (K == 0) ? TX : TY;     // nodes along the sweep
            constexpr int TC = (K == 0) ? TY : TX;     // lines of the sweep
            constexpr int NEL = TL + 6;
            constexpr int NS = TL + 4;
            // metrics of direction K on the lines of this sweep
            for (int q = t; q < NEL * TC; q += NT) {
                const int lx = (K == 0) ? q % NEL : 3 + q % TC;
                const int ly = (K == 0) ? 3 + q / NEL : q / TC;
                const int gx = ox + lx - 3, gy = oy + ly - 3;
                if (gx >= nx + 3 || gy >= ny + 3) continue;
                const long gi = gidx(gx, gy);
                const int li = lidx(lx, ly);
                S.m[0][li] = jxt ? 0.5 * jxt[(long)K * P + gi] : 0.0;
#pragma unroll
                for (int j = 0; j < D; j++) S.m[1 + j][li] = 0.5 * jxx[(long)(K * D + j) * P + gi];
            }
            __syncthreads();
            // line c of the sweep is row oy + c (K = 0) or column ox + c (K = 1);
            // node l of a line sits at patch along-coordinate l
            auto tidx = [](int l, int c) { return (K == 0) ? (l + NEX * (c + 3)) : ((c + 3) + NEX * l); };
            auto xidx = [](int s, int c) { return s + NS * c; };
            R (*X)[NS * TC] = reinterpret_cast<R (*)[NS * TC]>(&Xbuf[0]);
            const int nK = (K == 0) ? nx : ny, nL = (K == 0) ? ny : nx;
            const int o_along = (K == 0) ? ox : oy, o_line = (K == 0) ? oy : ox;
            const int fi = t % (TL + 1), fc = t / (TL + 1);
            // the interface's right stencil node fi + 5 (patch coordinate) must be loaded
            const bool f_ok = (t < (TL + 1) * TC) && (o_line + fc < nL) && (o_along + fi + 2 < nK + 3);
            // the acoustic and species fields in two groups in both
            // precisions: the region's right-hand sides stay in registers
            // across the two sweeps, and the FP32 kernel then fits three
            // waves per SIMD (2.0 ms against 2.65 ms per stage)
            interface_fluxes<N, D, NN, TL, TC, false, RC, R, 2>(ph, S, X, tidx, xidx,
                                                [&](int c) { return o_line + c < nL; }, fi, fc, f_ok,
                                                t - (int)((blockIdx.x + w) % NW) * 64);
            if (t < TX * TY) {
                const int lo = (K == 0) ? ni : nj, c = (K == 0) ? nj : ni;
                if (o_along + lo < nK && o_line + c < nL) {
                    const int l = lo + 3;
                    double gcl = 0.0;
#pragma unroll
                    for (int m = 1; m <= 3; m++)
                        gcl += ph.alpha[m - 1] * (S.m[0][tidx(l + m, c)] - S.m[0][tidx(l - m, c)]);
                    const double h = g.idxi[K];
                    // each direction's term is rounded on its own before it is
                    // added (separate statements, no fused multiply-add), as in
                    // the single-instance sweeps
                    const double dJ = -gcl * h;   // S.m holds half the metrics
                    accJ = accJ + dJ;
#pragma unroll
                    for (int cc = 0; cc < NC; cc++) {
                        const double d = -(double)(X[cc][xidx(lo + 2, c)] - X[cc][xidx(lo + 1, c)]) * h;
                        acc[cc] = acc[cc] + d;
                    }
                }
            }
            __syncthreads();   // S.m and X are reused by the next sweep / region
        };
        sweep(std::integral_constant<int, 0>{});
        sweep(std::integral_constant<int, 1>{});

        // ---- Shu-Osher combination, written to the node and its ghost images
        if (t < TX * TY && ox + ni < nx && oy + nj < ny) {
            const int gx = ox + ni, gy = oy + nj;
            const long gi = gidx(gx, gy);
            const double dt = dt_dev[bi];
            const double* __restrict__ JUn = tb.JUn[bi];
            const double* __restrict__ Jn = tb.Jn[bi];
            double* __restrict__ JUo = tb.JUo[bi];
            double* __restrict__ Jo = tb.Jo[bi];
            // stage 0 has ca = 0: the state at t^n is not read at all
            const bool rn = ca != 0.0;
            double o[NC];
#pragma unroll
            for (int cc = 0; cc < NC; cc++)
                o[cc] = ca * (rn ? JUn[cc * P + gi] : 0.0) + cb * (JUs[cc * P + gi] + dt * acc[cc]);
            const double oJ = ca * (rn ? Jn[gi] : 0.0) + cb * (Js[gi] + dt * accJ);
#pragma unroll
            for (int ky = -1; ky <= 1; ky++) {
                const int yy = gy + ky * ny;
                if (yy < -ng || yy >= ny + ng) continue;
#pragma unroll
                for (int kx = -1; kx <= 1; kx++) {
                    const int xx = gx + kx * nx;
                    if (xx < -ng || xx >= nx + ng) continue;
                    const long gj = gidx(xx, yy);
#pragma unroll
                    for (int cc = 0; cc < NC; cc++) JUo[cc * P + gj] = o[cc];
                    Jo[gj] = oJ;
                }
            }
        }
    }
    if (bad) atomicOr(status, bad);
}

// the region shapes of the autotuner's search: (TX, TY, threads); every
// sweep of a shape has at most as many interfaces as threads
#define ES_BATCH_SHAPES(X) X(0, 10, 10, 128) X(1, 15, 15, 256) X(2, 16, 15, 256) X(3, 15, 16, 256) \
                           X(4, 18, 13, 256) X(5, 21, 21, 512)

int batch_nshapes() { return 6; }

void batch_shape(int v, int* tx, int* ty, int* nt)
{
#define ES_SHAPE(V_, TX_, TY_, NT_) if (v == V_) { *tx = TX_; *ty = TY_; *nt = NT_; return; }
    ES_BATCH_SHAPES(ES_SHAPE)
#undef ES_SHAPE
    *tx = *ty = *nt = 0;
}

template <int N, typename R, int RC>
static hipError_t launch_variant(int v, const Phys& ph, const Geo* geos, const BatchTiling& tl,
                                 const BatchTables& tb, double ca, double cb, const double* dt_dev,
                                 unsigned* status, hipStream_t s)
{
#define ES_BATCH_CASE(V_, TX_, TY_, NT_)                                                             \
    if (v == V_) {                                                                                   \
        hipLaunchKernelGGL((k_stage2d_batched<N, TX_, TY_, NT_, R, RC>), dim3(tl.blocks), dim3(NT_), 0, s, \
                           ph, geos, tl.tiles, tl.ntiles, tb, ca, cb, dt_dev, status);               \
        return hipGetLastError();                                                                    \
    }
    ES_BATCH_SHAPES(ES_BATCH_CASE)
#undef ES_BATCH_CASE
    return hipErrorInvalidValue;
}

template <int N, typename R, int RC>
static hipError_t occupancy_variant(int v, int* blocks_per_cu)
{
#define ES_OCC_CASE(V_, TX_, TY_, NT_)                                                               \
    if (v == V_)                                                                                     \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,                          \
                                                            k_stage2d_batched<N, TX_, TY_, NT_, R, RC>, NT_, 0);
    ES_BATCH_SHAPES(ES_OCC_CASE)
#undef ES_OCC_CASE
    return hipErrorInvalidValue;
}

hipError_t batch_occupancy(int nspec, int mixed, int recon, int v, int* blocks_per_cu)
{
    if (recon == 1) {   // classical WENO5: FP64 only
        if (mixed) return hipErrorInvalidValue;
        return nspec == 1 ? occupancy_variant<1, double, 1>(v, blocks_per_cu)
                          : occupancy_variant<2, double, 1>(v, blocks_per_cu);
    }
    if (nspec == 1)
        return mixed ? occupancy_variant<1, float, 0>(v, blocks_per_cu) : occupancy_variant<1, double, 0>(v, blocks_per_cu);
    return mixed ? occupancy_variant<2, float, 0>(v, blocks_per_cu) : occupancy_variant<2, double, 0>(v, blocks_per_cu);
}

hipError_t launch_stage_batched(const Phys& ph, const Geo* geos, int mixed, const BatchTiling& tl,
                                const BatchTables& tb, double ca, double cb, const double* dt_dev,
                                unsigned* status, hipStream_t s)
{
    if (tl.ntiles == 0) return hipSuccess;
    if (ph.recon == 1) {   // classical WENO5: FP64 only (checked at create)
        if (mixed) return hipErrorInvalidValue;
        return ph.nspec == 1 ? launch_variant<1, double, 1>(tl.v, ph, geos, tl, tb, ca, cb, dt_dev, status, s)
                             : launch_variant<2, double, 1>(tl.v, ph, geos, tl, tb, ca, cb, dt_dev, status, s);
    }
    if (ph.nspec == 1)
        return mixed ? launch_variant<1, float, 0>(tl.v, ph, geos, tl, tb, ca, cb, dt_dev, status, s)
                     : launch_variant<1, double, 0>(tl.v, ph, geos, tl, tb, ca, cb, dt_dev, status, s);
    return mixed ? launch_variant<2, float, 0>(tl.v, ph, geos, tl, tb, ca, cb, dt_dev, status, s)
                 : launch_variant<2, double, 0>(tl.v, ph, geos, tl, tb, ca, cb, dt_dev, status, s);
}

}  // namespace es
