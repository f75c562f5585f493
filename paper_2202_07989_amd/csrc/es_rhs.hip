// es_rhs.hip -- the semi-discrete right-hand side (Sections 3.1-3.4) and the
// fused SSP-RK3 stage (Section 5) on gfx950.
//
// k_rhs_dir is one launch per direction k; k_rhs_xy (below) builds the x and
// y directions of a 3D grid in one launch, and 3D stages take it and then
// the z sweep.  In k_rhs_dir a block of 256 threads owns a tile of TL
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

// The x and y directions of a 3D grid in one launch.  A block of 512
// threads owns a TX x TY tile of one z plane: it stages the node quantities
// of the tile plus a 3-node halo along x and y (a plus-shaped patch; the
// corners are never read) and the halved metrics of both directions in LDS
// once, then waves 0-3 build the x fluxes of the tile's TY rows and waves
// 4-7 the y fluxes of its TX columns at the same time, each with the
// interface scheme of interface_fluxes.  A node's output is the x
// difference plus the y difference, each rounded on its own as the two
// separate sweeps round them, so the sum equals the x-sweep-then-y-sweep
// accumulation bit for bit; the z sweep then adds its own term.  Against the
// two separate sweeps this loads 1.8 instead of 2.6 nodes per owned node and
// skips the accumulator's round trip through memory.  LDS: 70 KB at
// 16 x 15 with two species, two blocks (four waves per SIMD) per compute
// unit.
template <int N, int TX, int TY, typename R, int RC, int MG>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_rhs_xy(Phys ph, Geo g, const double* __restrict__ JU, const double* __restrict__ Jv,
         const double* __restrict__ jxx, const double* __restrict__ jxt, double* __restrict__ accU,
         double* __restrict__ accJ, const double* __restrict__ tdiv, unsigned* __restrict__ status)
{
    constexpr int D = 3;
    constexpr int NT = 512;
    constexpr int NC = N + D + 1;
    constexpr int NEX = TX + 6, NEY = TY + 6;
    constexpr int NN = NEX * NEY;
    constexpr int XSX = (TX + 4) * TY, XSY = (TY + 4) * TX;    // exchange slots per component
    constexpr int XS = XSX > XSY ? XSX : XSY;
    static_assert((TX + 1) * TY <= NT / 2 && (TY + 1) * TX <= NT / 2 && 3 * TX <= 64 && 3 * TY <= 64,
                  "tile does not fit the block");
    __shared__ NodeTile<N, D, NN> S;     // S.m: the x metrics
    __shared__ double My[D + 1][NN];     // the y metrics
    static_assert(sizeof(R) * 2 * NC * XS <= sizeof(S) - sizeof(S.m), "exchange does not fit the tile");
    R (*Xb)[XS] = reinterpret_cast<R (*)[XS]>(&S.rho[0][0]);   // x rows 0..NC-1, y rows NC..2NC-1

    const long P = g.P;
    const int ng = g.ng, np0 = g.np[0], np1 = g.np[1];
    const int nx = g.n[0], ny = g.n[1];
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    const int ox = bx * TX, oy = by * TY;
    // padded index of patch node (0, 0), at interior (ox - 3, oy - 3) of plane bz
    const long base = ((long)(ng + bz) * np1 + (oy + ng - 3)) * np0 + (ox + ng - 3);
    const int t = threadIdx.x;

    // ---- node quantities and metrics of the patch -------------------------
    unsigned bad = 0;
    for (int q = t; q < NN; q += NT) {
        const int lx = q % NEX, ly = q / NEX;
        const bool cx = lx >= 3 && lx < 3 + TX, cy = ly >= 3 && ly < 3 + TY;
        if (!(cx || cy)) continue;                                        // corners
        if (ox + lx - 3 + ng >= np0 || oy + ly - 3 + ng >= np1) continue;  // beyond a ragged tile
        bad |= node_state<N, D, NN>(ph, S, q, JU, Jv, P, base + (long)ly * np0 + lx);
    }
    if (bad) atomicOr(status, bad);
    const double itd = tdiv ? 1.0 / *tdiv : 1.0;
    for (int q = t; q < NEX * TY + TX * NEY; q += NT) {
        const bool ydir = q >= NEX * TY;
        const int u = ydir ? q - NEX * TY : q;
        const int lx = ydir ? 3 + u % TX : u % NEX;
        const int ly = ydir ? u / TX : 3 + u / NEX;
        if (ox + lx - 3 + ng >= np0 || oy + ly - 3 + ng >= np1) continue;
        const long gi = base + (long)ly * np0 + lx;
        const int K = ydir ? 1 : 0;
        double (*Mk)[NN] = ydir ? My : S.m;
        const int li = lx + NEX * ly;
        Mk[0][li] = jxt ? 0.5 * (jxt[(long)K * P + gi] * itd) : 0.0;
#pragma unroll
        for (int j = 0; j < D; j++) Mk[1 + j][li] = 0.5 * jxx[(long)(K * D + j) * P + gi];
    }
    __syncthreads();

    // ---- interface fluxes: x in waves 0-3, y in waves 4-7 ------------------
    // x: interface fi of row fc (along-fastest, so a wave reads consecutive
    // nodes of a row); y: interface fi of column fc (column-fastest).  The
    // direction is uniform over a wave; read from the first lane, everything
    // derived from it lives in scalar registers
    const bool ydir = __builtin_amdgcn_readfirstlane(t / (NT / 2)) != 0;
    const int u = t & (NT / 2 - 1);
    const int TL = ydir ? TY : TX, TC = ydir ? TX : TY;
    const int fi = ydir ? u / TX : u % (TX + 1);
    const int fc = ydir ? u % TX : u / (TX + 1);
    const int o_along = ydir ? oy : ox, o_line = ydir ? ox : oy;
    const int n_line = ydir ? nx : ny, np_along = ydir ? np1 : np0;
    const bool f_ok = (u < (TL + 1) * TC) && (o_line + fc < n_line) && (o_along + fi + 2 + ng < np_along);
    // one copy of the arithmetic for both directions, the tile strides,
    // metric array and exchange rows picked per wave (compiling each
    // direction's arithmetic on its own under a branch took 4 % longer: the
    // join spills registers)
    const int sl = ydir ? NEX : 1, sc = ydir ? 1 : NEX, l0 = ydir ? 3 : 3 * NEX;
    const int xl = ydir ? TX : 1, xc = ydir ? 1 : TX + 4;
    interface_fluxes_m<N, D, NN, XS, true, RC, R, MG>(
        ph, S, ydir ? My : S.m, ydir ? Xb + NC : Xb, [=](int l, int c) { return l0 + l * sl + c * sc; },
        [=](int s, int c) { return s * xl + c * xc; }, [=](int c) { return o_line + c < n_line; }, fi, fc,
        f_ok, u - (int)(blockIdx.x & 3) * 64, TL, TC);

    // ---- node outputs: x difference + y difference -------------------------
    if (t < TX * TY) {
        const int ni = t % TX, nj = t / TX;
        if (ox + ni < nx && oy + nj < ny) {
            const long gi = base + (long)(nj + 3) * np0 + (ni + 3);
            auto lx_ = [](int l, int c) { return l + NEX * (c + 3); };
            auto ly_ = [](int l, int c) { return (c + 3) + NEX * l; };
            double gx = 0.0, gy = 0.0;
#pragma unroll
            for (int m = 1; m <= 3; m++) {
                gx += ph.alpha[m - 1] * (S.m[0][lx_(ni + 3 + m, nj)] - S.m[0][lx_(ni + 3 - m, nj)]);
                gy += ph.alpha[m - 1] * (My[0][ly_(nj + 3 + m, ni)] - My[0][ly_(nj + 3 - m, ni)]);
            }
            const double hx = g.idxi[0], hy = g.idxi[1];
            const R (*Xx)[XS] = Xb;
            const R (*Xy)[XS] = Xb + NC;
#pragma unroll
            for (int cc = 0; cc < NC; cc++) {
                const double dx = -(double)(Xx[cc][(ni + 2) + (TX + 4) * nj] - Xx[cc][(ni + 1) + (TX + 4) * nj]) * hx;
                const double dy = -(double)(Xy[cc][ni + TX * (nj + 2)] - Xy[cc][ni + TX * (nj + 1)]) * hy;
                accU[cc * P + gi] = dx + dy;
            }
            const double dJx = -gx * hx;   // S.m and My hold half the metrics
            const double dJy = -gy * hy;
            accJ[gi] = dJx + dJy;
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

// the x and y directions of a 3D grid in one launch (k_rhs_xy)
template <int N, typename R, int RC, int MG>
static hipError_t launch_xy(const Phys& ph, const Geo& g, const double* JU, const double* J,
                            const double* jxx, const double* jxt, double* accU, double* accJ,
                            const double* tdiv, unsigned* status, hipStream_t s)
{
    constexpr int TX = 16, TY = 15;
    const long gx = (g.n[0] + TX - 1) / TX, gy = (g.n[1] + TY - 1) / TY, gz = g.n[2];
    if (g.ng < 3 || gx * gy * gz > 0x7fffffffL || gy > 65535 || gz > 65535) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_rhs_xy<N, TX, TY, R, RC, MG>), dim3((unsigned)gx, (unsigned)gy, (unsigned)gz), dim3(512), 0, s,
                       ph, g, JU, J, jxx, jxt, accU, accJ, tdiv, status);
    return hipGetLastError();
}

template <int N, int D, typename R, int RC>
static hipError_t rhs_all(const Phys& ph, const Geo& g, const double* JU, const double* J,
                          const double* jxx, const double* jxt, double* outU, double* outJ,
                          const RkArgs* rk, unsigned* status, hipStream_t s)
{
    RkArgs none{nullptr, nullptr, nullptr, 0.0, 0.0};
    if (rk) none.tdiv = rk->tdiv;
    // 3D: x and y in one launch, then the z sweep (bitwise the three sweeps'
    // result, in both precisions; two field groups in the dissipation, which
    // keeps the FP32 launch at 90 registers)
    if constexpr (D == 3) {
        hipError_t e = launch_xy<N, R, RC, 2>(ph, g, JU, J, jxx, jxt, outU, outJ, none.tdiv, status, s);
        if (e != hipSuccess) return e;
        if (rk) return launch_dir<N, D, 2, MODE_RK, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, *rk, status, s);
        return launch_dir<N, D, 2, MODE_ADD, R, RC>(ph, g, JU, J, jxx, jxt, outU, outJ, none, status, s);
    } else {
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
