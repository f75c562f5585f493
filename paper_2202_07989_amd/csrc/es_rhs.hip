// es_rhs.hip -- the semi-discrete right-hand side (Sections 3.1-3.4) and the
// fused SSP-RK3 stage (Section 5) on gfx950.
//
// One launch per direction k.  A block of 256 threads owns a tile of TL
// nodes along k on TC grid lines (consecutive in the line ordering, so the
// fastest other index runs along the lines and global loads coalesce),
// stages the node quantities of the tile plus a 3-node halo along k in LDS,
// and builds the full numerical flux at each of the TL + 1 interfaces of
// every line, one thread per interface:
//   F_{i+1/2} = sum_m alpha_m sum_{s<m} F(i-s, i-s+m)  -  D_{i+1/2}
// (the interface form of eq ECFlux_curv_2p minus the ES dissipation
// 1/2 s T^T R Y [[W]]^WENO of eq HOstable).  Each two-point flux
// F(a, a+m) is evaluated once, by the thread whose interface has left node
// a; the m interfaces that use it collect it through an LDS exchange in
// three barrier-separated steps.  The node update is then the interface
// difference plus the GCL term delta_k[n_t] (eq GCL_flux), times -1/dxi_k,
// accumulated into the output; the last direction's epilogue can apply the
// Shu-Osher stage combination.
#include "es_flux.hpp"

namespace es {

// waves per SIMD: four for the FP64 x and y sweeps, whose dissipation takes
// the acoustic and species fields in two groups to stay within 128
// registers; three for the FP64 z sweep (its strided loads gain less from a
// fourth wave than its spills cost) and for FP32 (one group: splitting it
// costs more than a fourth wave gains)
template <int N, int D, int K, int TL, int TC, int MODE, typename R, int RC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((sizeof(R) == 8 && K != 2) ? 4 : 3, 8)))
k_rhs_dir(Phys ph, Geo g, const double* __restrict__ JU, const double* __restrict__ Jv,
          const double* __restrict__ jxx, const double* __restrict__ jxt,
          double* __restrict__ accU, double* __restrict__ accJ, RkArgs rk,
          unsigned* __restrict__ status)
{
    constexpr int NT = 256;
    constexpr int NC = N + D + 1;
    constexpr int NL = TL + 6;          // nodes per line: tile + 3-node halo on each side
    constexpr int NN = NL * TC;
    constexpr int NI = (TL + 1) * TC;   // interfaces (one thread each)
    constexpr int NS = TL + 4;          // exchange slots per line
    constexpr int NX = NS * TC;
    static_assert(NI <= NT && 3 * TC <= 64 && TL * TC <= NT, "tile does not fit the block");
    constexpr int FA = (K == 0) ? 1 : 0;   // across index that runs fastest
    constexpr int SA = (K == 2) ? 1 : 2;   // slowest across index
    __shared__ NodeTile<N, D, NN> S;
    // the flux exchange overlays the node quantities (not the metrics, which
    // the GCL term reads afterwards): 37 KB of LDS in all for two species in
    // 3D, so four blocks share a compute unit
    static_assert(sizeof(R) * NC * NX <= sizeof(S) - sizeof(S.m), "exchange does not fit the tile");
    R (*X)[NX] = reinterpret_cast<R (*)[NX]>(&S.rho[0][0]);

    const long P = g.P;
    const int nK = g.n[K];
    const int nF = g.n[FA];
    const long nlines = (long)nF * ((SA < D) ? g.n[SA] : 1);
    const int nseg = (nK + TL - 1) / TL;
    const int seg0 = (int)(blockIdx.x % nseg) * TL;
    const long line0 = (long)(blockIdx.x / nseg) * TC;
    const long sK = dir_stride(g, K);
    const int t = threadIdx.x;

    // LDS layouts are line-fastest in every direction, so the lanes of a wave
    // (consecutive lines) read consecutive words; the x sweep still walks x
    // fastest in its global loads and stores
    auto lidx = [](int l, int c) { return c + TC * l; };
    auto xidx = [](int s, int c) { return c + TC * s; };
    // padded index of the node at along-index 0 of each line of the block,
    // tabulated once (the line index splits into the two across indices by a
    // division)
    __shared__ long s_base[TC];
    if (t < TC) {
        const int L = (int)line0 + t;
        int i[3];
        i[K] = 0;
        i[FA] = g.ng + L % nF;
        i[SA] = (SA < D) ? g.ng + L / nF : 0;
        s_base[t] = node_index(g, i[0], i[1], i[2]);
    }
    __syncthreads();

    // ---- phase 1: node quantities of the tile (+ halo) into LDS ----------
    unsigned bad = 0;
    const double itd = rk.tdiv ? 1.0 / *rk.tdiv : 1.0;
    for (int q = t; q < NN; q += NT) {
        const int l = (K == 0) ? (q % NL) : (q / TC);
        const int c = (K == 0) ? (q / NL) : (q % TC);
        const int along = g.ng + seg0 + l - 3;
        if (along >= g.np[K] || line0 + c >= nlines) continue;
        const long gi = s_base[c] + along * sK;
        const int li = lidx(l, c);
        bad |= node_state<N, D, NN>(ph, S, li, JU, Jv, P, gi);
        S.m[0][li] = jxt ? 0.5 * (jxt[(long)K * P + gi] * itd) : 0.0;
#pragma unroll
        for (int j = 0; j < D; j++) S.m[1 + j][li] = 0.5 * jxx[(long)(K * D + j) * P + gi];
    }
    if (bad) atomicOr(status, bad);
    __syncthreads();

    // ---- phase 2: interface fluxes --------------------------------------
    const int fi = t / TC;
    const int fc = t % TC;
    // node fi + 5 must be inside the padded grid (ragged last segment)
    const bool f_ok = (t < NI) && (line0 + fc < nlines) && (g.ng + seg0 + fi + 2 < g.np[K]);
    interface_fluxes<N, D, NN, TL, TC, true, RC, R>(ph, S, X, lidx, xidx,
                                          [&](int c) { return line0 + c < nlines; }, fi, fc, f_ok,
                                          t - (int)(blockIdx.x & 3) * 64);

    // ---- phase 3: interface differences at the tile's nodes --------------
    const double dt = (MODE == MODE_RK) ? *rk.dt : 0.0;
    if (t < TL * TC) {
        const int lo = (K == 0) ? (t % TL) : (t / TC);
        const int c = (K == 0) ? (t / TL) : (t % TC);
        if (seg0 + lo < nK && line0 + c < nlines) {
            const int l = lo + 3;
            double gcl = 0.0;
#pragma unroll
            for (int m = 1; m <= 3; m++)
                gcl += ph.alpha[m - 1] * (S.m[0][lidx(l + m, c)] - S.m[0][lidx(l - m, c)]);
            const long gi = s_base[c] + (g.ng + seg0 + lo) * sK;
            const double h = g.idxi[K];
            const double dJ = -gcl * h;   // S.m holds half the metrics
#pragma unroll
            for (int cc = 0; cc < NC; cc++) {
                const double d = -(double)(X[cc][xidx(lo + 2, c)] - X[cc][xidx(lo + 1, c)]) * h;
                double* o = accU + cc * P + gi;
                if constexpr (MODE == MODE_WRITE) {
                    *o = d;
                } else if constexpr (MODE == MODE_ADD) {
                    *o += d;
                } else {
                    const double L = *o + d;
                    double* w = (rk.outU ? rk.outU : accU) + cc * P + gi;
                    // stage 0 has a = 0: Q_n is not read at all
                    const double qn = rk.a != 0.0 ? rk.JUn[cc * P + gi] : 0.0;
                    *w = rk.a * qn + rk.b * (JU[cc * P + gi] + dt * L);
                }
            }
            if constexpr (MODE == MODE_WRITE) {
                accJ[gi] = dJ;
            } else if constexpr (MODE == MODE_ADD) {
                accJ[gi] += dJ;
            } else {
                const double L = accJ[gi] + dJ;
                const double qn = rk.a != 0.0 ? rk.Jn[gi] : 0.0;
                (rk.outJ ? rk.outJ : accJ)[gi] = rk.a * qn + rk.b * (Jv[gi] + dt * L);
            }
        }
    }
}

// --------------------------------------------------------------------------
// host-side launch
// --------------------------------------------------------------------------
template <int N, int D, int K, int MODE, typename R, int RC>
static hipError_t launch_dir(const Phys& ph, const Geo& g, const double* JU, const double* J,
                             const double* jxx, const double* jxt, double* accU, double* accJ,
                             const RkArgs& rk, unsigned* status, hipStream_t s)
{
    // tile: TL nodes along k on TC lines.  The x sweep reads its lines along
    // the contiguous index, so a longer tile (24 on 10 lines: 250 interfaces)
    // cuts its halo re-reads (30/24 instead of 22/16 loaded per owned node,
    // -11% time); the y and z sweeps read rows of TC consecutive x values
    // across their lines, so they keep 15 lines (120-byte rows) of 16 nodes
    constexpr int TL = (K == 0) ? 24 : 16;
    constexpr int TC = (K == 0) ? 10 : 15;
    constexpr int FA = (K == 0) ? 1 : 0;
    constexpr int SA = (K == 2) ? 1 : 2;
    const long nseg = (g.n[K] + TL - 1) / TL;
    const long nlines = (long)g.n[FA] * ((SA < D) ? g.n[SA] : 1);
    const long nblk = nseg * ((nlines + TC - 1) / TC);
    if (nblk > 0x7fffffffL || nlines + TC > 0x7fffffffL) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)nblk);
    hipLaunchKernelGGL((k_rhs_dir<N, D, K, TL, TC, MODE, R, RC>), grid, dim3(256), 0, s, ph, g, JU, J,
                       jxx, jxt, accU, accJ, rk, status);
    return hipGetLastError();
}

template <int N, int D, typename R, int RC>
static hipError_t rhs_all(const Phys& ph, const Geo& g, const double* JU, const double* J,
                          const double* jxx, const double* jxt, double* outU, double* outJ,
                          const RkArgs* rk, unsigned* status, hipStream_t s)
{
    RkArgs none{nullptr, nullptr, nullptr, 0.0, 0.0};
    if (rk) none.tdiv = rk->tdiv;
    hipError_t e = launch_dir<N, D, 0, MODE_WRITE, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, none,
                                                      status, s);
    if (e != hipSuccess) return e;
    if constexpr (D == 2) {
        if (rk) return launch_dir<N, D, 1, MODE_RK, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, *rk, status, s);
        return launch_dir<N, D, 1, MODE_ADD, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, none, status, s);
    } else {
        e = launch_dir<N, D, 1, MODE_ADD, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, none, status, s);
        if (e != hipSuccess) return e;
        if (rk) return launch_dir<N, D, 2, MODE_RK, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, *rk, status, s);
        return launch_dir<N, D, 2, MODE_ADD, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, none, status, s);
    }
}

hipError_t launch_rhs(const Phys& ph, const Geo& g, int mixed, const double* JU, const double* J,
                      const double* jxx, const double* jxt, double* outU, double* outJ,
                      const RkArgs* rk, unsigned* status, hipStream_t s)
{
#define ES_RHS_CASE(NN_, DD_)                                                                          \
    if (ph.nspec == NN_ && g.dim == DD_) {                                                             \
        if (ph.recon == 1) {   /* classical WENO5: FP64 only (checked at create) */                 \
            if (mixed) return hipErrorInvalidValue;                                                    \
            return rhs_all<NN_, DD_, double, 1>(ph, g, JU, J, jxx, jxt, outU, outJ, rk, status, s);   \
        }                                                                                              \
        if (mixed) return rhs_all<NN_, DD_, float, 0>(ph, g, JU, J, jxx, jxt, outU, outJ, rk, status, s); \
        return rhs_all<NN_, DD_, double, 0>(ph, g, JU, J, jxx, jxt, outU, outJ, rk, status, s);       \
    }
    ES_RHS_CASE(1, 2)
    ES_RHS_CASE(2, 2)
    ES_RHS_CASE(1, 3)
    ES_RHS_CASE(2, 3)
#undef ES_RHS_CASE
    return hipErrorInvalidValue;
}

}  // namespace es
