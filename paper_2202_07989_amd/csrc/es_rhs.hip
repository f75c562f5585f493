// es_rhs.hip -- the semi-discrete right-hand side (Sections 3.1-3.4) and the
// fused SSP-RK3 stage (Section 5) on gfx950.
//
// One launch per direction k.  A block owns a tile of TL nodes along k by
// TC lines across it (lines adjacent along the fastest other index, so
// global loads are coalesced), stages the node quantities of the tile plus a
// 3-node halo along k in LDS, and then
//   phase 2: one thread per interface i+1/2 builds the ES dissipation
//            1/2 s T^T R Y [[W]]^WENO (eq HOstable) and parks it in LDS;
//   phase 3: one thread per node forms the 2w-order EC flux difference in
//            flux-differencing form sum_m alpha_m [F(i,i+m) - F(i-m,i)]
//            (the telescoped eq ECFlux_curv_2p), the GCL term delta_k[n_t]
//            (eq GCL_flux), subtracts the dissipation difference and
//            accumulates -(...)/dxi_k into the output.
// The last direction's epilogue can apply the Shu-Osher stage combination.
#include "es_kernels.hpp"

namespace es {

enum { MODE_WRITE = 0, MODE_ADD = 1, MODE_RK = 2 };

template <int N, int D, int NN>
struct NodeTile {
    double rho[N][NN];     // species densities
    double lrho[N][NN];    // their logs
    double lrt[NN];        // log of total density (N = 2)
    double gm[N == 2 ? NN : 1];   // mixture Gamma (N = 2)
    double rm[N == 2 ? NN : 1];   // mixture gas constant (N = 2)
    double v[D][NN];       // velocity
    double b[NN];          // beta = 1/T
    double lb[NN];         // log beta
    double p[NN];          // pressure
    double m[D + 1][NN];   // metrics of direction k: n_t, n_1..n_D
};

// two-point EC flux between tile nodes ia, ib (eq ECfluxMM), written in the
// direction-generic form n_t Utilde + sum_j n_j Ftilde_j:
//   M_l = {rho_l}^ln ({v}.n + n_t),  p^ = sum R_l {rho_l} / {beta} - p_inf,
//   momentum = {v} sum M_l + p^ n,
//   energy = sum M_l (c_vl/{beta}^ln - {|v|^2}/2) + {v}.momentum
//            + p_inf ({v}.n + n_t),
// with {|v|^2} the mean of squares.
template <int N, int D, int NN, typename R>
__device__ __forceinline__ void ec_pair(const Phys& ph, const NodeTile<N, D, NN>& S, int ia, int ib,
                                        R* F)
{
    constexpr int NC = N + D + 1;
    const R nt = R(0.5) * (R(S.m[0][ia]) + R(S.m[0][ib]));
    R n[D], vm[D];
    R vn = nt, v2 = R(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
        n[j] = R(0.5) * (R(S.m[1 + j][ia]) + R(S.m[1 + j][ib]));
        const R va = R(S.v[j][ia]), vb = R(S.v[j][ib]);
        vm[j] = R(0.5) * (va + vb);
        v2 += va * va + vb * vb;
        vn += vm[j] * n[j];
    }
    v2 *= R(0.5);
    const R ibln = R(inv_logmean(S.b[ia], S.b[ib], S.lb[ia], S.lb[ib]));
    const R bsum = R(S.b[ia]) + R(S.b[ib]);
    R Mt = R(0), Rr = R(0), eng = R(0);
#pragma unroll
    for (int l = 0; l < N; l++) {
        const R rln = R(logmean(S.rho[l][ia], S.rho[l][ib], S.lrho[l][ia], S.lrho[l][ib]));
        const R Ml = rln * vn;
        F[l] = Ml;
        Mt += Ml;
        Rr += R(ph.Rg[l]) * (R(S.rho[l][ia]) + R(S.rho[l][ib]));
        eng += Ml * (R(ph.cv[l]) * ibln - R(0.5) * v2);
    }
    const R phat = Rr / bsum - R(ph.pinf_tot);   // sum R_l {rho_l} / {beta} - p_inf
#pragma unroll
    for (int j = 0; j < D; j++) {
        const R fm = vm[j] * Mt + phat * n[j];
        F[N + j] = fm;
        eng += vm[j] * fm;
    }
    F[NC - 1] = eng + R(ph.pinf_tot) * vn;
}

// ES dissipation 1/2 s T^T R Y [[W]]^WENO at the interface between tile
// nodes iL (= i) and iR (= i+1); st[t] are the tile indices of nodes
// i-2..i+3.  Interface metrics, averages and R follow Section 3.4.
template <int N, int D, int NN, typename R>
__device__ __forceinline__ void dissipation(const Phys& ph, const NodeTile<N, D, NN>& S,
                                            const int st[6], const Weno<R>& Wc, R* Dout)
{
    constexpr int NC = N + D + 1;
    const int iL = st[2], iR = st[3];
    // interface metric: mean of the two nodes
    R n[D];
    const R nt = R(0.5) * (R(S.m[0][iL]) + R(S.m[0][iR]));
    R nn2 = R(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
        n[j] = R(0.5) * (R(S.m[1 + j][iL]) + R(S.m[1 + j][iR]));
        nn2 += n[j] * n[j];
    }
    const R nn = sqrt(nn2);
    const R inn = nn > R(0) ? R(1) / nn : R(0);
    Rot<D, R> T;
    if (nn > R(0)) {
        make_rot<D, R>(n, inn, T);
    } else {
#pragma unroll
        for (int a = 0; a < D; a++)
#pragma unroll
            for (int b = 0; b < D; b++) T.t[a][b] = R(a == b);
    }
    // averaged state
    R vbar[D];
    R vn = R(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
        vbar[j] = R(0.5) * (R(S.v[j][iL]) + R(S.v[j][iR]));
        vn += vbar[j] * n[j];
    }
    Frame<N, D, R> F;
    rot_apply<D, R>(T, vbar, F.vh);
    R vv = R(0);
#pragma unroll
    for (int j = 0; j < D; j++) vv += F.vh[j] * F.vh[j];
    F.K = R(0.5) * vv;
    const R Tbar = R(inv_logmean(S.b[iL], S.b[iR], S.lb[iL], S.lb[iR]));   // 1/{beta}^ln
    if constexpr (N == 1) {
        const R G = R(ph.gam[0]), Rg = R(ph.Rg[0]), cv = R(ph.cv[0]);
        const R rho = R(logmean(S.rho[0][iL], S.rho[0][iR], S.lrho[0][iL], S.lrho[0][iR]));
        F.c = sqrt(G * Rg * Tbar);
        F.H = G * cv * Tbar + F.K;
        F.sa = sqrt(rho / (R(2) * G * Rg));
        F.se = sqrt(rho / (cv * G));
        F.st = sqrt(rho * Tbar);
    } else {
        R rl[2];
        const R Rm[2] = {R(S.rm[iL]), R(S.rm[iR])};
        const R Gm[2] = {R(S.gm[iL]), R(S.gm[iR])};
#pragma unroll
        for (int l = 0; l < 2; l++)
            rl[l] = R(logmean(S.rho[l][iL], S.rho[l][iR], S.lrho[l][iL], S.lrho[l][iR]));
        const double rL = S.rho[0][iL] + S.rho[1][iL], rR = S.rho[0][iR] + S.rho[1][iR];
        const R rho = R(logmean(rL, rR, S.lrt[iL], S.lrt[iR]));
        const R Rb = R(0.5) * (Rm[0] + Rm[1]);
        const R Gb = R(0.5) * (Gm[0] + Gm[1]);
        const R irho = R(1) / rho;
        R rhoh = R(0.5) * (R(S.p[iL]) + R(S.p[iR]));
#pragma unroll
        for (int l = 0; l < 2; l++) rhoh += R(ph.cv[l]) * rl[l] * Tbar + R(ph.pinf[l]);
        F.H = rhoh * irho + F.K;
        F.Y[0] = rl[0] * irho;
        F.Y[1] = rl[1] * irho;
        const R igm1 = R(1) / (Gb - R(1));
#pragma unroll
        for (int l = 0; l < 2; l++)
            F.e2[l] = F.K - (R(ph.cv[l]) + R(ph.Rg[l]) - Gb * R(ph.cv[l])) * Tbar * igm1;
        F.c = sqrt(Gb * Rb * Tbar);
        F.sq = sqrt(rho / (Gb * Rb));
        F.s2a = F.sq * R(0.70710678118654752440);
        const R yy = sqrt(F.Y[0] * F.Y[1]);
        const R sg = sqrt(Gb - R(1));
        const R r21 = R(ph.r21);
        F.d11 = -F.sq * yy * sqrt(Gb * r21);
        F.d12 = F.sq * F.Y[0] * sg;
        F.d21 = F.sq * yy * sqrt(Gb / r21);
        F.d22 = F.sq * F.Y[1] * sg;
    }
    const R s = fabs(nt + vn) + nn * F.c;

    // scaled entropy variables W_j = R^T T V(U_j), j = i-2..i+3
    R W[6][NC];
#pragma unroll
    for (int t = 0; t < 6; t++) {
        const int q = st[t];
        const R bq = R(S.b[q]);
        R vq[D], vr[D];
        R v2 = R(0);
#pragma unroll
        for (int j = 0; j < D; j++) {
            vq[j] = R(S.v[j][q]);
            v2 += vq[j] * vq[j];
        }
        R y[NC];
        const double lbq = S.lb[q];
#pragma unroll
        for (int l = 0; l < N; l++)
            y[l] = R(ph.cv[l] * lbq + ph.Rg[l] * S.lrho[l][q] + ph.cvgam[l]) - R(0.5) * bq * v2;
        rot_apply<D, R>(T, vq, vr);
#pragma unroll
        for (int j = 0; j < D; j++) y[N + j] = bq * vr[j];
        y[NC - 1] = -bq;
        frame_project<N, D, R>(F, y, W[t]);
    }
    // MR-WENO on each scaled characteristic field, sign matrix Y
    R Z[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const R wm = mr5<R>(W[0][c], W[1][c], W[2][c], W[3][c], W[4][c], Wc);
        const R wp = mr5<R>(W[5][c], W[4][c], W[3][c], W[2][c], W[1][c], Wc);
        const R jw = wp - wm;
        const R jump = W[3][c] - W[2][c];
        // sign matrix Y: the WENO jump and the jump agree in sign, and the jump
        // is not zero to working precision (across a contact the acoustic
        // jumps vanish up to rounding; those count as sign 0)
        const bool y = (jw * jump > R(0)) && (fabs(jump) > Wc.zero_tol * (fabs(W[2][c]) + fabs(W[3][c])));
        Z[c] = y ? jw : R(0);
    }
    R RZ[NC];
    frame_expand<N, D, R>(F, Z, RZ);
    const R hs = R(0.5) * s;
#pragma unroll
    for (int l = 0; l < N; l++) Dout[l] = hs * RZ[l];
    R mv[D], mo[D];
#pragma unroll
    for (int j = 0; j < D; j++) mv[j] = RZ[N + j];
    rot_apply_t<D, R>(T, mv, mo);
#pragma unroll
    for (int j = 0; j < D; j++) Dout[N + j] = hs * mo[j];
    Dout[NC - 1] = hs * RZ[NC - 1];
}

template <int N, int D, int K, int TL, int TC, int MODE, typename R>
__global__ void __launch_bounds__(256)
k_rhs_dir(Phys ph, Geo g, const double* __restrict__ JU, const double* __restrict__ Jv,
          const double* __restrict__ jxx, const double* __restrict__ jxt,
          double* __restrict__ accU, double* __restrict__ accJ, RkArgs rk,
          unsigned* __restrict__ status)
{
    constexpr int NC = N + D + 1;
    constexpr int NL = TL + 6;
    constexpr int NN = NL * TC;
    constexpr int NI = (TL + 1) * TC;
    constexpr int FA = (K == 0) ? 1 : 0;   // across index that runs fastest
    constexpr int SA = (K == 2) ? 1 : 2;   // slowest across index
    __shared__ NodeTile<N, D, NN> S;
    __shared__ R sD[NC][NI];

    const long P = g.P;
    const int nK = g.n[K];
    const int nF = g.n[FA];
    const int nseg = (nK + TL - 1) / TL;
    const int seg = blockIdx.x % nseg;
    const int fc = blockIdx.x / nseg;
    const int seg0 = seg * TL, c0 = fc * TC;
    const int slow = (SA < D) ? (int)blockIdx.y + g.ng : 0;

    auto lidx = [](int l, int c) { return (K == 0) ? (l + NL * c) : (c + TC * l); };
    auto gidx = [&](int along, int fast) -> long {
        int i[3];
        i[K] = along;
        i[FA] = fast;
        i[SA] = slow;
        return node_index(g, i[0], i[1], i[2]);
    };

    // ---- phase 1: node quantities of the tile (+ halo) into LDS ----------
    unsigned bad = 0;
    for (int t = threadIdx.x; t < NN; t += blockDim.x) {
        const int l = (K == 0) ? (t % NL) : (t / TC);
        const int c = (K == 0) ? (t / NL) : (t % TC);
        const int along = g.ng + seg0 + l - 3;
        if (along >= g.np[K] || c0 + c >= nF) continue;
        const long gi = gidx(along, g.ng + c0 + c);
        const int li = lidx(l, c);
        const double Jq = Jv[gi];
        const double iJ = 1.0 / Jq;
        double U[NC];
#pragma unroll
        for (int cc = 0; cc < NC; cc++) U[cc] = JU[cc * P + gi] * iJ;
        double rt = 0.0, cvr = 0.0, rR = 0.0;
#pragma unroll
        for (int s = 0; s < N; s++) {
            rt += U[s];
            cvr += ph.cv[s] * U[s];
            rR += ph.Rg[s] * U[s];
        }
        const double ir = 1.0 / rt;
        double kin = 0.0;
#pragma unroll
        for (int j = 0; j < D; j++) {
            const double vj = U[N + j] * ir;
            S.v[j][li] = vj;
            kin += 0.5 * U[N + j] * vj;
        }
        const double e = U[NC - 1] - kin - ph.pinf_tot;
        const double T = e / cvr;
        const double beta = cvr / e;
        S.b[li] = beta;
        S.lb[li] = log(beta);
        S.p[li] = rR * T - ph.pinf_tot;
        bool ok = (T > 0.0) && isfinite(T) && isfinite(kin);
#pragma unroll
        for (int s = 0; s < N; s++) {
            S.rho[s][li] = U[s];
            S.lrho[s][li] = log(U[s]);
            ok = ok && (U[s] > 0.0);
        }
        if constexpr (N == 2) {
            double cg = 0.0;
#pragma unroll
            for (int q = 0; q < N; q++) cg += ph.cvgam[q] * U[q];
            S.lrt[li] = log(rt);
            S.gm[li] = cg / cvr;
            S.rm[li] = rR * ir;
        }
        if (!ok) bad |= 1u;
        if (!(Jq > 0.0)) bad |= 2u;
        S.m[0][li] = jxt ? jxt[(long)K * P + gi] : 0.0;
#pragma unroll
        for (int j = 0; j < D; j++) S.m[1 + j][li] = jxx[(long)(K * D + j) * P + gi];
    }
    if (bad) atomicOr(status, bad);
    __syncthreads();

    // ---- phase 2: interface dissipation --------------------------------
    if (ph.dissipation) {
        Weno<R> Wc;
        Wc.chi1 = R(ph.chi[0]); Wc.chi2 = R(ph.chi[1]); Wc.chi3 = R(ph.chi[2]);
        Wc.eps = R(ph.eps); Wc.ichi3 = R(ph.ichi3); Wc.c1c3 = R(ph.c1c3); Wc.c2c3 = R(ph.c2c3);
        Wc.zero_tol = sizeof(R) == 8 ? R(1e-12) : R(4e-6);
        for (int t = threadIdx.x; t < NI; t += blockDim.x) {
            const int li = (K == 0) ? (t % (TL + 1)) : (t / TC);   // interface slot 0..TL
            const int c = (K == 0) ? (t / (TL + 1)) : (t % TC);
            const int l = li + 2;                                   // left node of the interface
            if (g.ng + seg0 + l >= g.np[K] || c0 + c >= nF) continue;  // node l+3 not loaded
            int st[6];
#pragma unroll
            for (int q = 0; q < 6; q++) st[q] = lidx(l - 2 + q, c);
            R Dv[NC];
            dissipation<N, D, NN, R>(ph, S, st, Wc, Dv);
            const int di = (K == 0) ? (li + (TL + 1) * c) : (c + TC * li);
#pragma unroll
            for (int cc = 0; cc < NC; cc++) sD[cc][di] = Dv[cc];
        }
        __syncthreads();
    }

    // ---- phase 3: flux differences at the tile's nodes -------------------
    const double dt = (MODE == MODE_RK) ? *rk.dt : 0.0;
    for (int t = threadIdx.x; t < TL * TC; t += blockDim.x) {
        const int lo = (K == 0) ? (t % TL) : (t / TC);
        const int c = (K == 0) ? (t / TL) : (t % TC);
        if (seg0 + lo >= nK || c0 + c >= nF) continue;
        const int l = lo + 3;
        const int me = lidx(l, c);
        R acc[NC];
#pragma unroll
        for (int cc = 0; cc < NC; cc++) acc[cc] = R(0);
        double gcl = 0.0;
#pragma unroll
        for (int m = 1; m <= 3; m++) {
            if (m > ph.w) break;
            const R am = R(ph.alpha[m - 1]);
            const int ip = lidx(l + m, c), imn = lidx(l - m, c);
            R Fp[NC], Fm[NC];
            ec_pair<N, D, NN, R>(ph, S, me, ip, Fp);
            ec_pair<N, D, NN, R>(ph, S, imn, me, Fm);
#pragma unroll
            for (int cc = 0; cc < NC; cc++) acc[cc] += am * (Fp[cc] - Fm[cc]);
            gcl += ph.alpha[m - 1] * (S.m[0][ip] - S.m[0][imn]);
        }
        if (ph.dissipation) {
            const int dr = (K == 0) ? (lo + 1 + (TL + 1) * c) : (c + TC * (lo + 1));
            const int dl = (K == 0) ? (lo + (TL + 1) * c) : (c + TC * lo);
#pragma unroll
            for (int cc = 0; cc < NC; cc++) acc[cc] -= sD[cc][dr] - sD[cc][dl];
        }
        const long gi = gidx(g.ng + seg0 + lo, g.ng + c0 + c);
        const double h = g.idxi[K];
        const double dJ = -0.5 * gcl * h;
#pragma unroll
        for (int cc = 0; cc < NC; cc++) {
            const double d = -(double)acc[cc] * h;
            double* o = accU + cc * P + gi;
            if constexpr (MODE == MODE_WRITE) {
                *o = d;
            } else if constexpr (MODE == MODE_ADD) {
                *o += d;
            } else {
                const double L = *o + d;
                *o = rk.a * rk.JUn[cc * P + gi] + rk.b * (JU[cc * P + gi] + dt * L);
            }
        }
        if constexpr (MODE == MODE_WRITE) {
            accJ[gi] = dJ;
        } else if constexpr (MODE == MODE_ADD) {
            accJ[gi] += dJ;
        } else {
            const double L = accJ[gi] + dJ;
            accJ[gi] = rk.a * rk.Jn[gi] + rk.b * (Jv[gi] + dt * L);
        }
    }
}

// --------------------------------------------------------------------------
// host-side launch
// --------------------------------------------------------------------------
template <int N, int D, int K, int MODE, typename R>
static hipError_t launch_dir(const Phys& ph, const Geo& g, const double* JU, const double* J,
                             const double* jxx, const double* jxt, double* accU, double* accJ,
                             const RkArgs& rk, unsigned* status, hipStream_t s)
{
    constexpr int TL = 16, TC = 16;
    constexpr int FA = (K == 0) ? 1 : 0;
    constexpr int SA = (K == 2) ? 1 : 2;
    const int nseg = (g.n[K] + TL - 1) / TL;
    const int nfc = (g.n[FA] + TC - 1) / TC;
    const int nslow = (SA < D) ? g.n[SA] : 1;
    dim3 grid(nseg * nfc, nslow);
    hipLaunchKernelGGL((k_rhs_dir<N, D, K, TL, TC, MODE, R>), grid, dim3(256), 0, s, ph, g, JU, J,
                       jxx, jxt, accU, accJ, rk, status);
    return hipGetLastError();
}

template <int N, int D, typename R>
static hipError_t rhs_all(const Phys& ph, const Geo& g, const double* JU, const double* J,
                          const double* jxx, const double* jxt, double* outU, double* outJ,
                          const RkArgs* rk, unsigned* status, hipStream_t s)
{
    RkArgs none{nullptr, nullptr, nullptr, 0.0, 0.0};
    hipError_t e = launch_dir<N, D, 0, MODE_WRITE, R>(ph, g, JU, J, jxx, jxt, outU, outJ, none,
                                                      status, s);
    if (e != hipSuccess) return e;
    if constexpr (D == 2) {
        if (rk) return launch_dir<N, D, 1, MODE_RK, R>(ph, g, JU, J, jxx, jxt, outU, outJ, *rk, status, s);
        return launch_dir<N, D, 1, MODE_ADD, R>(ph, g, JU, J, jxx, jxt, outU, outJ, none, status, s);
    } else {
        e = launch_dir<N, D, 1, MODE_ADD, R>(ph, g, JU, J, jxx, jxt, outU, outJ, none, status, s);
        if (e != hipSuccess) return e;
        if (rk) return launch_dir<N, D, 2, MODE_RK, R>(ph, g, JU, J, jxx, jxt, outU, outJ, *rk, status, s);
        return launch_dir<N, D, 2, MODE_ADD, R>(ph, g, JU, J, jxx, jxt, outU, outJ, none, status, s);
    }
}

hipError_t launch_rhs(const Phys& ph, const Geo& g, int mixed, const double* JU, const double* J,
                      const double* jxx, const double* jxt, double* outU, double* outJ,
                      const RkArgs* rk, unsigned* status, hipStream_t s)
{
#define ES_RHS_CASE(NN_, DD_)                                                                     \
    if (ph.nspec == NN_ && g.dim == DD_) {                                                        \
        if (mixed) return rhs_all<NN_, DD_, float>(ph, g, JU, J, jxx, jxt, outU, outJ, rk, status, s); \
        return rhs_all<NN_, DD_, double>(ph, g, JU, J, jxx, jxt, outU, outJ, rk, status, s);     \
    }
    ES_RHS_CASE(1, 2)
    ES_RHS_CASE(2, 2)
    ES_RHS_CASE(1, 3)
    ES_RHS_CASE(2, 3)
#undef ES_RHS_CASE
    return hipErrorInvalidValue;
}

}  // namespace es
