// es_flux.hpp -- the per-node and per-interface pieces of the ES flux
// (Sections 3.1-3.4) shared by the direction-sweep kernels of es_rhs.hip and
// the batched stage kernel of es_batch.hip.  Node quantities live in an LDS
// tile (NodeTile); the functions read them by tile index.
#pragma once
#include "es_kernels.hpp"

namespace es {

enum { MODE_WRITE = 0, MODE_ADD = 1, MODE_RK = 2 };

template <int N, int D, int NN>
struct NodeTile {
    double rho[N][NN];     // species densities
    double lrho[N][NN];    // their logs
    double lrt[N == 2 ? NN : 1];  // log of the total density (N = 2)
    double v[D][NN];       // velocity
    double b[NN];          // beta = 1/T
    double lb[NN];         // log beta
    float ay[NN];          // sum_l |y_l| (species entropy variables), and
    float av[NN];          // beta |v|_1: row magnitudes for the sign test's zero tolerance
    double m[D + 1][NN];   // half the metrics of direction k: n_t/2, n_1/2..n_D/2 (an
                           // interface average is then one sum; halving is exact)
};

// mixture Gamma, gas constant and pressure of tile node q (N = 2)
template <int N, int D, int NN>
__device__ __forceinline__ void mixture(const Phys& ph, const NodeTile<N, D, NN>& S, int q,
                                        double& gm, double& rm, double& p)
{
    const double r0 = S.rho[0][q], r1 = S.rho[1][q];
    const double cvr = ph.cv[0] * r0 + ph.cv[1] * r1;
    const double rR = ph.Rg[0] * r0 + ph.Rg[1] * r1;
    gm = (ph.cvgam[0] * r0 + ph.cvgam[1] * r1) * rcp(cvr);
    rm = rR * rcp(r0 + r1);
    p = rR * rcp(S.b[q]) - ph.pinf_tot;
}

// two-point EC flux between tile nodes ia, ib (eq ECfluxMM), written in the
// direction-generic form n_t Utilde + sum_j n_j Ftilde_j:
//   M_l = {rho_l}^ln ({v}.n + n_t),  p^ = Pi - p_inf with Pi = sum R_l {rho_l} / {beta},
//   momentum = {v} sum M_l + p^ n,
//   energy = sum M_l (c_vl/{beta}^ln - {|v|^2}/2) + |{v}|^2 sum M_l + Pi {v}.n + p_inf n_t,
// with {|v|^2} the mean of squares.  The energy line is {v}.momentum +
// p_inf ({v}.n + n_t) with the two p_inf {v}.n terms cancelled by hand, and
// Pi is formed in FP64 in both precisions: with a stiffened gas Pi and
// p_inf are both ~p_inf, so neither difference may be left to FP32.
// (M: the halved metrics of the direction, indexed like the tile)
template <int N, int D, int NN, typename R>
__device__ __forceinline__ void ec_pair(const Phys& ph, const NodeTile<N, D, NN>& S, const double (*M)[NN],
                                        int ia, int ib, R* F)
{
    constexpr int NC = N + D + 1;
    const R nt = R(M[0][ia]) + R(M[0][ib]);
    R n[D], vm[D];
    R vdn = R(0), v2 = R(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
        n[j] = R(M[1 + j][ia]) + R(M[1 + j][ib]);
        const R va = R(S.v[j][ia]), vb = R(S.v[j][ib]);
        vm[j] = R(0.5) * (va + vb);
        v2 += va * va + vb * vb;
        vdn += vm[j] * n[j];
    }
    v2 *= R(0.5);
    const R vn = vdn + nt;
    const R ibln = R(inv_logmean(S.b[ia], S.b[ib], S.lb[ia], S.lb[ib]));
    double Rr = 0.0;
#pragma unroll
    for (int l = 0; l < N; l++) Rr += ph.Rg[l] * (S.rho[l][ia] + S.rho[l][ib]);
    const double Pi = Rr * rcp(S.b[ia] + S.b[ib]);
    const R phat = R(Pi - ph.pinf_tot);
    R Mt = R(0), eng = R(0);
#pragma unroll
    for (int l = 0; l < N; l++) {
        const R rln = R(logmean(S.rho[l][ia], S.rho[l][ib], S.lrho[l][ia], S.lrho[l][ib]));
        const R Ml = rln * vn;
        F[l] = Ml;
        Mt += Ml;
        eng += Ml * (R(ph.cv[l]) * ibln - R(0.5) * v2);
    }
    R vv = R(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
        F[N + j] = vm[j] * Mt + phat * n[j];
        vv += vm[j] * vm[j];
    }
    F[NC - 1] = eng + vv * Mt + R(Pi) * vdn + R(ph.pinf_tot) * nt;
}

// ES dissipation 1/2 s T^T R Y [[W]]^WENO at the interface between tile
// nodes iL (= i) and iR (= i+1); st[t] are the tile indices of nodes
// i-2..i+3.  Interface metrics, averages and R follow Section 3.4.  MG: the
// acoustic and species fields in one group or two.
template <int N, int D, int NN, int RC, typename R, int MG>
__device__ __forceinline__ void dissipation(const Phys& ph, const NodeTile<N, D, NN>& S, const double (*M)[NN],
                                            const int st[6], const Weno<R>& Wc, R* Dout)
{
    constexpr int NC = N + D + 1;
    const int iL = st[2], iR = st[3];
    // interface metric: mean of the two nodes
    R n[D];
    const R nt = R(M[0][iL]) + R(M[0][iR]);
    R nn2 = R(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
        n[j] = R(M[1 + j][iL]) + R(M[1 + j][iR]);
        nn2 += n[j] * n[j];
    }
    const bool nz = nn2 > R(0);
    const R inn = nz ? rsqrt_pos(nn2) : R(0);
    const R nn = nn2 * inn;
    Rot<D, R> T;
    make_rot<D, R>(n, inn, nz, T);
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
        F.c = sqrt_pos(G * Rg * Tbar);
        F.H = G * cv * Tbar + F.K;
        F.sa = sqrt_pos(rho * rcp(R(2) * G * Rg));
        F.se = sqrt_pos(rho * rcp(cv * G));
        F.st = sqrt_pos(rho * Tbar);
    } else {
        R rl[2];
        double gmL, gmR, rmL, rmR, pL, pR;
        mixture<N, D, NN>(ph, S, iL, gmL, rmL, pL);
        mixture<N, D, NN>(ph, S, iR, gmR, rmR, pR);
        const R Rm[2] = {R(rmL), R(rmR)};
        const R Gm[2] = {R(gmL), R(gmR)};
#pragma unroll
        for (int l = 0; l < 2; l++)
            rl[l] = R(logmean(S.rho[l][iL], S.rho[l][iR], S.lrho[l][iL], S.lrho[l][iR]));
        const double rL = S.rho[0][iL] + S.rho[1][iL], rR = S.rho[0][iR] + S.rho[1][iR];
        const R rho = R(logmean(rL, rR, S.lrt[iL], S.lrt[iR]));
        const R Rb = R(0.5) * (Rm[0] + Rm[1]);
        const R Gb = R(0.5) * (Gm[0] + Gm[1]);
        const R irho = rcp(rho);
        R rhoh = R(0.5) * (R(pL) + R(pR));
#pragma unroll
        for (int l = 0; l < 2; l++) rhoh += R(ph.cv[l]) * rl[l] * Tbar + R(ph.pinf[l]);
        F.H = rhoh * irho + F.K;
        F.Y[0] = rl[0] * irho;
        F.Y[1] = rl[1] * irho;
        const R igm1 = rcp(Gb - R(1));
#pragma unroll
        for (int l = 0; l < 2; l++)
            F.e2[l] = F.K - (R(ph.cv[l]) + R(ph.Rg[l]) - Gb * R(ph.cv[l])) * Tbar * igm1;
        F.c = sqrt_pos(Gb * Rb * Tbar);
        F.sq = sqrt_pos(rho * rcp(Gb * Rb));
        F.s2a = F.sq * R(0.70710678118654752440);
        const R yy = sqrt_pos(F.Y[0] * F.Y[1]);
        const R sg = sqrt_pos(Gb - R(1));
        const R syg = F.sq * yy * sqrt_pos(Gb);
        F.d11 = -syg * R(ph.sr21);
        F.d12 = F.sq * F.Y[0] * sg;
        F.d21 = syg * R(ph.isr21);
        F.d22 = F.sq * F.Y[1] * sg;
    }
    const R s = fabs(nt + vn) + nn * F.c;

    // scaled entropy variables W_j = R^T T V(U_j) of the stencil nodes
    // j = i-2..i+3, one group of characteristic fields at a time (the
    // tangential fields, then the acoustic and species fields, these two in
    // separate groups when MG = 2), each group's MR-WENO jumps taken as soon
    // as its stencil values exist.  The acoustic
    // and species fields see the rotated momentum variables only through
    // (T vbar).(T b v) = b vbar.v and the normal row of T v.
    R Z[NC];
    // MR-WENO on one scaled characteristic field, sign matrix Y: the WENO
    // jump and the jump agree in sign, and the jump is not zero to working
    // precision, i.e. above zero_tol times mag, a bound on the size of the
    // terms that make W_i and W_{i+1}: max_l |R_lc| sum_l |y_l| over the
    // species rows, plus sum_e |R_ec| a_e with a_e = beta |v|_1 (>= every
    // rotated |y_{N+j}|) for the momentum rows and beta for the energy row,
    // all summed over nodes i and i+1.  Across a contact the acoustic jumps vanish up to rounding, in an
    // isentropic flow the entropy field's do; those count as sign 0.
    auto weno_field = [&](const R (&w)[6], R mag) -> R {
        R jump;
        const R jw = mr5_jump<R, RC == 1>(w[0], w[1], w[2], w[3], w[4], w[5], Wc, jump);
        const bool y = (jw * jump > R(0)) && (fabs(jump) > Wc.zero_tol * mag);
        return y ? jw : R(0);
    };
    // row magnitudes of nodes i and i+1, summed (the node part of the zero
    // tolerance, kept per node in the tile): ay = sum_l |y_l|, av = beta
    // |v|_1, aE = beta
    auto node_scales = [&](R& ay, R& av, R& aE) {
        ay = R(S.ay[iL]) + R(S.ay[iR]);
        av = R(S.av[iL]) + R(S.av[iR]);
        aE = R(fabs(S.b[iL]) + fabs(S.b[iR]));
    };
    asm volatile("" ::: "memory");
    {
        R Wt[D - 1][6];
        const R sct = (N == 1) ? F.st : F.sq * F.c;   // scale of the tangential columns
#pragma unroll
        for (int t = 0; t < 6; t++) {
            const int q = st[t];
            const R bq = R(S.b[q]);
            R vq[D], vr[D];
#pragma unroll
            for (int j = 0; j < D; j++) vq[j] = R(S.v[j][q]);
            rot_apply<D, R>(T, vq, vr);
            R yt[D - 1];
#pragma unroll
            for (int j = 1; j < D; j++) yt[j - 1] = bq * vr[j];
            R wt[D - 1];
            frame_project_tan<N, D, R>(F, yt, -bq, wt);
#pragma unroll
            for (int j = 0; j < D - 1; j++) Wt[j][t] = wt[j];
        }
        R ay, av, aE;
        node_scales(ay, av, aE);
        R mt[D - 1];
        bool need = false;
#pragma unroll
        for (int j = 0; j < D - 1; j++) {
            mt[j] = sct * (av + fabs(F.vh[j + 1]) * aE);
            need = need || fabs(Wt[j][3] - Wt[j][2]) > Wc.zero_tol * mt[j];
        }
        // where no lane of the wave has a jump above the tolerance, every
        // field of the group has Y = 0 and its WENO jump is not needed (the
        // same for the second group)
        if (__any(need)) {
#pragma unroll
            for (int j = 0; j < D - 1; j++) Z[N + 1 + j] = weno_field(Wt[j], mt[j]);
        } else {
#pragma unroll
            for (int j = 0; j < D - 1; j++) Z[N + 1 + j] = R(0);
        }
    }
    // the acoustic and species (entropy) fields, as one group or (MG = 2)
    // two, the acoustic fields and then the species fields, each reloading
    // its node values from LDS rather than keeping the previous group's loads
    // live across its WENO: fewer registers for more loads
    {
        constexpr int NM = N + 2;                  // main fields 0..N and NC - 1
        constexpr int NGRP = MG;
        R mg[NM];
        {
            R ay, av, aE;
            node_scales(ay, av, aE);
            frame_scale_main<N, D, R>(F, ay, av, aE, mg);
        }
#pragma unroll
        for (int grp = 0; grp < NGRP; grp++) {
            asm volatile("" ::: "memory");
            // main field of the c-th member of this group, and its slot in Z
            const int nf = NGRP == 1 ? NM : (grp == 0 ? 2 : NM - 2);
            auto mfield = [&](int c) { return NGRP == 1 ? c : (grp == 0 ? (c == 0 ? 0 : NM - 1) : 1 + c); };
            auto zslot = [&](int m) { return m <= N ? m : NC - 1; };
            R Wg[NM][6];
#pragma unroll
            for (int t = 0; t < 6; t++) {
                const int q = st[t];
                const R bq = R(S.b[q]);
                R vq[D], vr[D];
                R v2 = R(0), vbv = R(0);
#pragma unroll
                for (int j = 0; j < D; j++) {
                    vq[j] = R(S.v[j][q]);
                    v2 += vq[j] * vq[j];
                    vbv += vbar[j] * vq[j];
                }
                R ys[N];
                const double lbq = S.lb[q];
#pragma unroll
                for (int l = 0; l < N; l++)
                    ys[l] = R(ph.cv[l] * lbq + ph.Rg[l] * S.lrho[l][q] + ph.cvgam[l]) - R(0.5) * bq * v2;
                rot_apply<D, R>(T, vq, vr);
                R wm[NM];
                frame_project_main<N, D, R>(F, ys, bq * vr[0], bq * vbv, -bq, wm);
#pragma unroll
                for (int c = 0; c < NM; c++)
                    if (c < nf) Wg[c][t] = wm[mfield(c)];
            }
            bool need = false;
#pragma unroll
            for (int c = 0; c < NM; c++)
                if (c < nf) need = need || fabs(Wg[c][3] - Wg[c][2]) > Wc.zero_tol * mg[mfield(c)];
            if (__any(need)) {
#pragma unroll
                for (int c = 0; c < NM; c++)
                    if (c < nf) Z[zslot(mfield(c))] = weno_field(Wg[c], mg[mfield(c)]);
            } else {
#pragma unroll
                for (int c = 0; c < NM; c++)
                    if (c < nf) Z[zslot(mfield(c))] = R(0);
            }
        }
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

// Numerical flux at the TL + 1 interfaces of each of TC lines of a tile
// (the interface form of eq ECFlux_curv_2p minus the ES dissipation of eq
// HOstable), left in X slot f + 1 of line c.
//
// Interface slot f = 0..TL of a line has left node l = f + 2 (the tile's
// first own node is l = 3).  Its thread evaluates P_m = F(l, l+m), m = 1..3,
// and with B(f) = a3 P_3 and H(f) = a2 P_2 + B(f) the flux is
//   F_f = a1 P_1 - D_f + H(f) + H(f-1) + B(f-2),
// so each two-point flux is evaluated once.  X slot f + 2 carries B(f),
// then H(f), and finally slot f + 1 holds F_f.  The pairs F(0,3), F(1,4),
// F(1,3) left of the first interface (B(-2), B(-1), H(-1)) are taken by
// the lanes with hid = 0 .. 3 TC - 1 (one wave, chosen by the caller).
// lidx(l, c) is the tile index of node l of line c, xidx(s, c) the X index
// of slot s of line c, line_ok(c) whether line c exists; f_ok says that
// this thread's interface (fi, fc) exists and its six nodes are loaded.
// RC selects the reconstruction of the dissipation (0: multi-resolution
// WENO, 1: classical WENO5).  With XALIAS, X overlays the node quantities of S (all but the metrics):
// every flux is then formed in registers first and X is written only after
// a barrier that ends all node reads.  Every thread of the block must call
// this (it holds barriers).
// (MG: the dissipation's acoustic and species fields in one group or two;
// two in FP64, where they keep the sweeps within fewer registers)
// interface_fluxes_m is the general form: the metrics M of the direction
// are passed in, X rows are XS slots long, and the tile's TL and TC may be
// run-time values (a block that sweeps two directions at once picks them per
// wave); interface_fluxes takes the tile's own metrics and fixed sizes.
template <int N, int D, int NN, int XS, bool XALIAS, int RC, typename R, int MG, typename LI, typename XI,
          typename LOK>
__device__ __forceinline__ void interface_fluxes_m(const Phys& ph, const NodeTile<N, D, NN>& S,
                                                   const double (*M)[NN], R (*X)[XS], LI lidx, XI xidx,
                                                   LOK line_ok, int fi, int fc, bool f_ok, int hid,
                                                   int TL, int TC)
{
    constexpr int NC = N + D + 1;
    const R a1 = R(ph.alpha[0]), a2 = R(ph.alpha[1]), a3 = R(ph.alpha[2]);
    const int fl = fi + 2;
    R G[NC], A2[NC], B3[NC];
    if (f_ok) {
        R F[NC];
        if (ph.dissipation) {
            // zero tolerance of the sign test, relative to the size of the
            // terms of W, in the precision of the arithmetic (0: the sign
            // test as printed)
            const Weno<R> Wc = make_weno<R>(ph.chi, ph.eps, sizeof(R) == 8 ? ph.stol64 : ph.stol32);
            int st[6];
#pragma unroll
            for (int q = 0; q < 6; q++) st[q] = lidx(fl - 2 + q, fc);
            dissipation<N, D, NN, RC, R, MG>(ph, S, M, st, Wc, G);
        } else {
#pragma unroll
            for (int cc = 0; cc < NC; cc++) G[cc] = R(0);
        }
        ec_pair<N, D, NN, R>(ph, S, M, lidx(fl, fc), lidx(fl + 1, fc), F);
#pragma unroll
        for (int cc = 0; cc < NC; cc++) G[cc] = a1 * F[cc] - G[cc];
        if (a2 != R(0)) {
            ec_pair<N, D, NN, R>(ph, S, M, lidx(fl, fc), lidx(fl + 2, fc), F);
        } else {
#pragma unroll
            for (int cc = 0; cc < NC; cc++) F[cc] = R(0);
        }
#pragma unroll
        for (int cc = 0; cc < NC; cc++) A2[cc] = a2 * F[cc];
        if (a3 != R(0)) {
            ec_pair<N, D, NN, R>(ph, S, M, lidx(fl, fc), lidx(fl + 3, fc), F);
        } else {
#pragma unroll
            for (int cc = 0; cc < NC; cc++) F[cc] = R(0);
        }
#pragma unroll
        for (int cc = 0; cc < NC; cc++) B3[cc] = a3 * F[cc];
    }
    // the pairs F(0,3), F(1,4), F(1,3) left of the first interface
    const bool halo = hid >= 0 && hid < 3 * TC;
    R Bh[NC];
    int hslot = 0, hc = 0;
    if (halo) {
        const int h = hid / TC;
        hc = hid % TC;
        const R am = (h == 2) ? a2 : a3;
        hslot = (h == 0) ? 0 : ((h == 1) ? 1 : TL + 3);
        if (line_ok(hc) && am != R(0)) {
            ec_pair<N, D, NN, R>(ph, S, M, lidx(h == 0 ? 0 : 1, hc), lidx(h == 1 ? 4 : 3, hc), Bh);
        } else {
#pragma unroll
            for (int cc = 0; cc < NC; cc++) Bh[cc] = R(0);
        }
#pragma unroll
        for (int cc = 0; cc < NC; cc++) Bh[cc] = am * Bh[cc];
    }
    if constexpr (XALIAS) __syncthreads();   // node reads end before X overwrites them
    if (halo) {
#pragma unroll
        for (int cc = 0; cc < NC; cc++) X[cc][xidx(hslot, hc)] = Bh[cc];
    }
    if (f_ok) {
#pragma unroll
        for (int cc = 0; cc < NC; cc++) X[cc][xidx(fi + 2, fc)] = B3[cc];
    }
    __syncthreads();
    R Hf[NC], Hm[NC];
    if (f_ok) {
#pragma unroll
        for (int cc = 0; cc < NC; cc++) {
            G[cc] += X[cc][xidx(fi, fc)];                   // + B(f-2)
            Hf[cc] = A2[cc] + X[cc][xidx(fi + 2, fc)];      // H(f)
        }
        if (fi == 0) {
#pragma unroll
            for (int cc = 0; cc < NC; cc++) Hm[cc] = X[cc][xidx(TL + 3, fc)] + X[cc][xidx(1, fc)];
        }
    }
    __syncthreads();
    if (f_ok) {
#pragma unroll
        for (int cc = 0; cc < NC; cc++) X[cc][xidx(fi + 2, fc)] = Hf[cc];
        if (fi == 0) {
#pragma unroll
            for (int cc = 0; cc < NC; cc++) X[cc][xidx(1, fc)] = Hm[cc];
        }
    }
    __syncthreads();
    if (f_ok) {
#pragma unroll
        for (int cc = 0; cc < NC; cc++) {
            const int xi = xidx(fi + 1, fc);
            X[cc][xi] = G[cc] + (Hf[cc] + X[cc][xi]);     // F_f into slot f+1
        }
    }
    __syncthreads();
}

template <int N, int D, int NN, int TL, int TC, bool XALIAS, int RC, typename R,
          int MG = (sizeof(R) == 8 ? 2 : 1), typename LI, typename XI, typename LOK>
__device__ __forceinline__ void interface_fluxes(const Phys& ph, const NodeTile<N, D, NN>& S,
                                                 R (*X)[(TL + 4) * TC], LI lidx, XI xidx,
                                                 LOK line_ok, int fi, int fc, bool f_ok, int hid)
{
    interface_fluxes_m<N, D, NN, (TL + 4) * TC, XALIAS, RC, R, MG>(ph, S, S.m, X, lidx, xidx, line_ok, fi, fc,
                                                                  f_ok, hid, TL, TC);
}

// primitive node quantities of node gi of (JU, J) into tile slot li; returns
// the status bits of the node (1: rho_l <= 0, T <= 0 or non-finite; 2: J <= 0)
template <int N, int D, int NN>
__device__ __forceinline__ unsigned node_state(const Phys& ph, NodeTile<N, D, NN>& S, int li,
                                               const double* __restrict__ JU,
                                               const double* __restrict__ Jv, long P, long gi)
{
    constexpr int NC = N + D + 1;
    const double Jq = Jv[gi];
    const double iJ = rcp(Jq);
    double U[NC];
#pragma unroll
    for (int cc = 0; cc < NC; cc++) U[cc] = JU[cc * P + gi] * iJ;
    double rt = 0.0, cvr = 0.0;
#pragma unroll
    for (int sp = 0; sp < N; sp++) {
        rt += U[sp];
        cvr += ph.cv[sp] * U[sp];
    }
    const double ir = rcp(rt);
    double kin = 0.0;
#pragma unroll
    for (int j = 0; j < D; j++) {
        const double vj = U[N + j] * ir;
        S.v[j][li] = vj;
        kin += 0.5 * U[N + j] * vj;
    }
    const double e = U[NC - 1] - kin - ph.pinf_tot;
    const double beta = cvr * rcp(e);
    S.b[li] = beta;
    const double lbeta = ln_pos(beta);
    S.lb[li] = lbeta;
    bool ok = (beta > 0.0) && isfinite(beta) && isfinite(kin);
    double v1 = 0.0, v2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; j++) {
        const double vj = S.v[j][li];
        v1 += fabs(vj);
        v2 += vj * vj;
    }
    double ysum = 0.0;
#pragma unroll
    for (int sp = 0; sp < N; sp++) {
        S.rho[sp][li] = U[sp];
        const double lr = ln_pos(U[sp]);
        S.lrho[sp][li] = lr;
        ysum += fabs(ph.cv[sp] * lbeta + ph.Rg[sp] * lr + ph.cvgam[sp] - 0.5 * beta * v2);
        ok = ok && (U[sp] > 0.0);
    }
    S.ay[li] = float(ysum);
    S.av[li] = float(fabs(beta) * v1);
    if constexpr (N == 2) S.lrt[li] = ln_pos(rt);
    unsigned bad = ok ? 0u : 1u;
    if (!(Jq > 0.0)) bad |= 2u;
    return bad;
}

}  // namespace es
