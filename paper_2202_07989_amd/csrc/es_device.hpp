// es_device.hpp -- device-side building blocks of the gfx950 path.
//
// Li, Duan & Tang, arXiv 2202.07989.  Everything here is evaluated per node
// or per interface inside the kernels of es_rhs.hip / es_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace es {

// --------------------------------------------------------------------------
// parameters passed by value to every kernel
// --------------------------------------------------------------------------
struct Phys {
    int nspec, dim, nc, w, dissipation;
    int recon;                // 0: multi-resolution WENO, 1: classical WENO5 (Jiang-Shu)
    double cv[2], gam[2], pinf[2], Rg[2], cvgam[2];
    double pinf_tot;
    double alpha[3];          // alpha_{w,m}
    double chi[3], eps;       // MR-WENO linear weights and epsilon
    double r21;               // R_2 / R_1 (N = 2)
    double sr21, isr21;       // sqrt(R_2 / R_1) and its reciprocal
    double stol64, stol32;    // zero tolerances of the sign matrix (FP64, FP32 arithmetic)
};

struct Geo {
    int dim, ng;
    int n[3];                 // interior nodes
    int np[3];                // padded extents
    long P;                   // points per component
    double dxi[3], idxi[3], len[3];
    int bc[3][2];             // face conditions (BC_*), [k][0] low face, [k][1] high face
    double wall[3][2];        // physical coordinate x_k of the non-periodic faces
};

enum { BC_PERIODIC = 0, BC_REFLECT = 1, BC_OUTFLOW = 2, BC_INFLOW = 3 };

__device__ __forceinline__ long node_index(const Geo& g, int i0, int i1, int i2)
{
    return ((long)i2 * g.np[1] + i1) * g.np[0] + i0;
}

__device__ __forceinline__ long dir_stride(const Geo& g, int k)
{
    return k == 0 ? 1L : (k == 1 ? (long)g.np[0] : (long)g.np[0] * g.np[1]);
}

// --------------------------------------------------------------------------
// reciprocal of a finite, normal, nonzero x: the hardware estimate refined
// by Newton steps r <- r (2 - x r) (two in FP64, one in FP32), within about
// an ulp of 1/x.  It replaces IEEE division on the hot path, whose scaling
// for special operands costs about twice the instructions; a zero, infinite
// or denormal x only arises from a non-physical state, which then turns
// non-finite and is reported by the status checks.
// --------------------------------------------------------------------------
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ float rcp(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// square root of a finite, positive, normal x: the hardware 1/sqrt estimate
// y, then s = x y, h = y/2 refined by one Goldschmidt step and two
// corrections s += (x - s^2) h, within about an ulp; IEEE sqrt adds the
// scaling of tiny operands and the selects for 0 and infinity
__device__ __forceinline__ double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double sq = x * y, h = 0.5 * y;
    const double r = fma(-h, sq, 0.5);
    sq = fma(sq, r, sq);
    h = fma(h, r, h);
    double d = fma(-sq, sq, x);
    sq = fma(d, h, sq);
    d = fma(-sq, sq, x);
    return fma(d, h, sq);
}

__device__ __forceinline__ float sqrt_pos(float x) { return sqrtf(x); }

// 1/sqrt(x) of a finite, positive, normal x: the hardware estimate refined by
// two Newton steps y <- y + y/2 (1 - x y^2)
__device__ __forceinline__ double rsqrt_pos(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// FP32 operands go through FP64: the FP32 estimate does not take denormal
// operands, and the squared tangential part of a nearly axis-aligned
// interface normal can be one
__device__ __forceinline__ float rsqrt_pos(float x) { return (float)rsqrt_pos((double)x); }

// natural logarithm of a finite, positive, normal x: x = 2^e m with m in
// [sqrt(1/2), sqrt(2)), ln x = e ln 2 + 2 atanh(s), s = (m - 1)/(m + 1),
// |s| <= 0.1716, and atanh(s) = s sum_k s^(2k)/(2k+1) taken to k = 9 (the
// first dropped term is below 1e-17 relative).  ln 2 is carried as a double
// and its remainder, each multiplied into a fused multiply-add.  Within two
// ulps (the rounding of m + 1 dominates near x = 1); a third of the
// instructions of the library logarithm, which works in double-double.
// Non-positive or non-finite x only arise from states the status checks
// report.
__device__ __forceinline__ double ln_pos(double x)
{
    int e = __builtin_amdgcn_frexp_exp(x);        // x = m 2^e, m in [1/2, 1)
    double m = __builtin_amdgcn_frexp_mant(x);
    const bool lo = m < 0.70710678118654752440;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double s = (m - 1.0) * rcp(m + 1.0);
    const double z = s * s;
    double p = 1.0 / 19.0;
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double hs = 2.0 * s;
    const double lm = fma(hs * z, p, hs);
    const double de = (double)e;
    return fma(de, 0x1.62e42fefa39efp-1, fma(de, 0x1.abc9e3b39803fp-56, lm));
}

// --------------------------------------------------------------------------
// logarithmic mean [[a]]/[[ln a]] (Section 3.3.1) from precomputed node logs.
// Near a = b (f = (a-b)/(a+b), u = f^2 < 1e-4) the ratio is evaluated from
// series in u instead: {a}^ln = (a+b)/2 * f/atanh(f) and
// 1/{a}^ln = 2/(a+b) * atanh(f)/f, each truncated after u^3 (the dropped
// terms are below 1e-17 relative there).  One division on either branch.
// --------------------------------------------------------------------------
__device__ __forceinline__ double logmean(double a, double b, double la, double lb)
{
    const double d = a - b, s = a + b;
    if (d * d < 1.0e-4 * (s * s)) {
        const double is = rcp(s);
        const double f = d * is, u = f * f;
        const double G = 1.0 - u * (1.0 / 3.0 + u * (4.0 / 45.0 + u * (44.0 / 945.0)));
        return 0.5 * s * G;
    }
    return d * rcp(la - lb);
}

__device__ __forceinline__ double inv_logmean(double a, double b, double la, double lb)
{
    const double d = a - b, s = a + b;
    if (d * d < 1.0e-4 * (s * s)) {
        const double is = rcp(s);
        const double f = d * is, u = f * f;
        const double F = 1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0)));
        return 2.0 * F * is;
    }
    return (la - lb) * rcp(d);
}

// --------------------------------------------------------------------------
// fifth-order multi-resolution WENO (Appendix A): value at the right face of
// the centre cell of (q_-2 .. q_2), written in the four differences
// D_0..D_3 = q_-1 - q_-2, q_0 - q_-1, q_1 - q_0, q_2 - q_1 (the scheme only
// ever looks at differences: the smoothness indicators are quadratic forms
// in them and every reconstruction is q_0 plus a combination of them):
//   beta_1 = min(D_1^2, D_2^2),
//   beta_2 = a_2^2 + 13/3 a_3^2 with a_2 = (D_1 + D_2)/2, a_3 = (D_2 - D_1)/2,
//   beta_3 = the printed closed form, with its Legendre coefficients
//            t_1 = (7 S12 - S03)/12, t_2 = (11 A03 + 163 A21)/260,
//            c_4 = (S03 - S12)/12, c_5 = -(A03 + 3 A21)/24
//            (S03 = D_0 + D_3, S12 = D_1 + D_2, A03 = D_0 - D_3, A21 = D_2 - D_1),
//   h_1 - q_0 = 0, h_2 - q_0 = (D_1 + 2 D_2)/6,
//   h_3 - q_0 = (-2 D_0 + 11 D_1 + 24 D_2 - 3 D_3)/60,
// and the value is q_0 + (w_2 (h_2 - q_0) + w_3 (hc - q_0)) / (w_1 + w_2 + w_3)
// with hc - q_0 = ((h_3 - q_0) - chi_2 (h_2 - q_0)) / chi_3.  These equal the
// Legendre forms exactly in rational arithmetic.  The weights
// w_m = chi_m (1 + tau / d_m), d_m = eps + beta_m, are taken over the common
// denominator d_1 d_2 d_3 as chi_m e_m with e_m = (d_m + tau) prod_{l!=m} d_l,
// and the linear weights are folded into the reconstructions:
//   num = e_2 c_2 + e_3 c_3,  den = sum chi_m e_m,
// with c_2 = chi_2 (h_2 - q_0) and c_3 = chi_3 (hc - q_0) = (h_3 - q_0) - c_2.
// --------------------------------------------------------------------------
template <typename R>
struct Weno {
    R chi1, chi2, chi3, eps;
    R zero_tol;           // relative size below which a jump counts as zero in the sign test
};

template <typename R>
__device__ __forceinline__ Weno<R> make_weno(const double chi[3], double eps, double zero_tol)
{
    Weno<R> W;
    W.chi1 = R(chi[0]); W.chi2 = R(chi[1]); W.chi3 = R(chi[2]); W.eps = R(eps);
    W.zero_tol = R(zero_tol);
    return W;
}

// numerator and denominator of (value - q_0)
template <typename R>
__device__ __forceinline__ void mr5_diff(R D0, R D1, R D2, R D3, const Weno<R>& W, R& num, R& den)
{
    const R S03 = D0 + D3, S12 = D1 + D2, A03 = D0 - D3, A21 = D2 - D1;
    const R b1 = fmin(D1 * D1, D2 * D2);
    const R b2 = R(0.25) * (S12 * S12) + R(13.0 / 12.0) * (A21 * A21);
    const R u1 = R(7) * S12 - S03, u2 = R(11) * A03 + R(163) * A21, u3 = S03 - S12, u4 = A03 + R(3) * A21;
    const R b3 = R(1.0 / 144.0) * (u1 * u1) + R(13.0 / 3.0 / 67600.0) * (u2 * u2)
               + R(781.0 / 20.0 / 144.0) * (u3 * u3) + R(1421461.0 / 2275.0 / 576.0) * (u4 * u4);
    R tau = fabs(b3 - b1) + fabs(b3 - b2);
    tau = R(0.25) * (tau * tau);
    const R c2 = W.chi2 * (R(1.0 / 6.0) * D1 + R(1.0 / 3.0) * D2);
    const R c3 = R(11.0 / 60.0) * D1 + R(0.4) * D2 - R(1.0 / 30.0) * D0 - R(0.05) * D3 - c2;
    R d1 = W.eps + b1, d2 = W.eps + b2, d3 = W.eps + b3;
    if constexpr (sizeof(R) == 4) {   // keep the products in float range
        const R dm = rcp(fmax(fmax(d1, d2), d3));
        d1 *= dm; d2 *= dm; d3 *= dm; tau *= dm;
    }
    const R e1 = (d1 + tau) * (d2 * d3);
    const R e2 = (d2 + tau) * (d1 * d3);
    const R e3 = (d3 + tau) * (d1 * d2);
    num = e2 * c2 + e3 * c3;
    den = W.chi1 * e1 + W.chi2 * e2 + W.chi3 * e3;
}

// Classical fifth-order WENO of Jiang and Shu (the comparison variant of
// Section 5) in the same difference form, value - q_0 = num / den:
//   candidates  c_0 = (5 D_1 - 2 D_0)/6, c_1 = (D_1 + 2 D_2)/6, c_2 = (4 D_2 - D_3)/6,
//   beta_0 = 13/12 (D_1 - D_0)^2 + 1/4 (3 D_1 - D_0)^2,
//   beta_1 = 13/12 (D_2 - D_1)^2 + 1/4 (D_1 + D_2)^2,
//   beta_2 = 13/12 (D_3 - D_2)^2 + 1/4 (3 D_2 - D_3)^2,
// weights d_k / e_k with e_k = (eps + beta_k)^2 and d = (1/10, 6/10, 3/10),
// taken over the common denominator e_0 e_1 e_2.
template <typename R>
__device__ __forceinline__ void js5_diff(R D0, R D1, R D2, R D3, R eps, R& num, R& den)
{
    const R s0 = D1 - D0, t0 = R(3) * D1 - D0;
    const R s1 = D2 - D1, t1 = D1 + D2;
    const R s2 = D3 - D2, t2 = R(3) * D2 - D3;
    R e0 = eps + (R(13.0 / 12.0) * (s0 * s0) + R(0.25) * (t0 * t0));
    R e1 = eps + (R(13.0 / 12.0) * (s1 * s1) + R(0.25) * (t1 * t1));
    R e2 = eps + (R(13.0 / 12.0) * (s2 * s2) + R(0.25) * (t2 * t2));
    e0 *= e0; e1 *= e1; e2 *= e2;
    if constexpr (sizeof(R) == 4) {   // keep the products in float range
        const R em = rcp(fmax(fmax(e0, e1), e2));
        e0 *= em; e1 *= em; e2 *= em;
    }
    const R p0 = R(0.1) * (e1 * e2), p1 = R(0.6) * (e0 * e2), p2 = R(0.3) * (e0 * e1);
    const R c0 = (R(5) * D1 - R(2) * D0) * R(1.0 / 6.0);
    const R c1 = (D1 + R(2) * D2) * R(1.0 / 6.0);
    const R c2 = (R(4) * D2 - D3) * R(1.0 / 6.0);
    num = p0 * c0 + p1 * c1 + p2 * c2;
    den = p0 + p1 + p2;
}

// Jump of the two one-sided reconstructions at an interface, wp - wm, from
// the stencil W_0..W_5 (nodes i-2..i+3): wm is the reconstruction of
// (W_0..W_4) at the right face of node i, wp that of the mirrored
// (W_5..W_1) at the left face of node i+1.  With D_k = W_{k+1} - W_k,
// wm = W_2 + Nm/Dm from (D_0, D_1, D_2, D_3) and wp = W_3 + Np/Dp from
// (-D_4, -D_3, -D_2, -D_1), so wp - wm = D_2 + Np/Dp - Nm/Dm; FP64 takes the
// two quotients over one denominator.  jump_out = W_3 - W_2 = D_2.
// JS selects the classical reconstruction instead of MR.
template <typename R, bool JS = false>
__device__ __forceinline__ R mr5_jump(R q0, R q1, R q2, R q3, R q4, R q5, const Weno<R>& W, R& jump_out)
{
    const R D0 = q1 - q0, D1 = q2 - q1, D2 = q3 - q2, D3 = q4 - q3, D4 = q5 - q4;
    R nm, dm, np, dp;
    if constexpr (JS) {
        js5_diff<R>(D0, D1, D2, D3, W.eps, nm, dm);
        js5_diff<R>(-D4, -D3, -D2, -D1, W.eps, np, dp);
    } else {
        mr5_diff<R>(D0, D1, D2, D3, W, nm, dm);
        mr5_diff<R>(-D4, -D3, -D2, -D1, W, np, dp);
    }
    jump_out = D2;
    if constexpr (sizeof(R) == 8) return D2 + (np * dm - nm * dp) * rcp(dp * dm);
    else return D2 + (np * rcp(dp) - nm * rcp(dm));
}

// --------------------------------------------------------------------------
// velocity-block rotation T (eq rotamatrix): first row n/|n|; tangential
// rows from theta = atan2(n2, n1) (0 when n1 = n2 = 0) and phi.
// --------------------------------------------------------------------------
template <int D, typename R>
struct Rot;
template <typename R>
struct Rot<2, R> {       // T = [[c, s], [-s, c]]
    R c, s;
};
template <typename R>
struct Rot<3, R> {       // T = [[cp ct, cp st, sp], [-st, ct, 0], [-sp ct, -sp st, cp]]
    R ct, st, cp, sp;
};

// T from the interface normal n, given 1/|n| (nonzero = false: n = 0, T = I)
template <int D, typename R>
__device__ __forceinline__ void make_rot(const R n[D], R inv_norm, bool nonzero, Rot<D, R>& T)
{
    if constexpr (D == 2) {
        T.c = nonzero ? n[0] * inv_norm : R(1);
        T.s = nonzero ? n[1] * inv_norm : R(0);
    } else {
        // the tangential part (n_1, n_2) and its length in FP64 in both
        // precisions: in FP32 its square can be denormal (a nearly
        // axis-aligned normal) and would carry only a few bits
        const double a = n[0], b = n[1];
        const double r12sq = a * a + b * b;
        T.ct = R(1); T.st = R(0); T.cp = R(1); T.sp = R(0);
        if (nonzero) {
            T.cp = R(0);
            if (r12sq > 0.0) {
                const double ir12 = rsqrt_pos(r12sq);
                T.ct = R(a * ir12);
                T.st = R(b * ir12);
                T.cp = R(r12sq * ir12) * inv_norm;
            }
            T.sp = n[2] * inv_norm;
        }
    }
}

// out = T in
template <int D, typename R>
__device__ __forceinline__ void rot_apply(const Rot<D, R>& T, const R in[D], R out[D])
{
    if constexpr (D == 2) {
        out[0] = T.c * in[0] + T.s * in[1];
        out[1] = T.c * in[1] - T.s * in[0];
    } else {
        const R a = T.ct * in[0] + T.st * in[1];
        out[0] = T.cp * a + T.sp * in[2];
        out[1] = T.ct * in[1] - T.st * in[0];
        out[2] = T.cp * in[2] - T.sp * a;
    }
}

// out = T^T in
template <int D, typename R>
__device__ __forceinline__ void rot_apply_t(const Rot<D, R>& T, const R in[D], R out[D])
{
    if constexpr (D == 2) {
        out[0] = T.c * in[0] - T.s * in[1];
        out[1] = T.s * in[0] + T.c * in[1];
    } else {
        const R b = T.cp * in[0] - T.sp * in[2];
        out[0] = T.ct * b - T.st * in[1];
        out[1] = T.st * b + T.ct * in[1];
        out[2] = T.sp * in[0] + T.cp * in[2];
    }
}

// --------------------------------------------------------------------------
// Scaled eigenvector frame at an interface (Section 3.4), in factored form
// R = Rtilde * S with Rtilde the unscaled right eigenvectors of the rotated
// averaged state and S the symmetric scaling (diagonal, plus the 2x2 species
// block D^Y for N = 2).  Only the entries that are not structurally zero or
// one are kept, so W = R^T (T V) and R z cost ~4 nc multiply-adds.
// --------------------------------------------------------------------------
template <int N, int D, typename R>
struct Frame {
    R vh[D];     // rotated averaged velocity
    R c;         // averaged sound speed
    R H;         // averaged total enthalpy
    R K;         // |v|^2 / 2
    R Y[2];      // N = 2: averaged mass fractions
    R e2[2];     // N = 2: K - d_l / (Gamma - 1)
    R sa, se, st; // N = 1: scalings of acoustic, entropy, tangential columns
    R s2a, sq;   // N = 2: sqrt(rho/(Gamma R))/sqrt(2) and sqrt(rho/(Gamma R))
    R d11, d12, d21, d22;  // N = 2: D^Y scaled by sqrt(rho/(Gamma R))
};

// W = R^T y (y = T V) split into the tangential fields, W_{N+t} for
// t = 1..D-1 from y_{N+t} and yE = y_{nc-1} ...
template <int N, int D, typename R>
__device__ __forceinline__ void frame_project_tan(const Frame<N, D, R>& F, const R* yt, R yE, R* Wt)
{
    const R sc = (N == 1) ? F.st : F.sq * F.c;
#pragma unroll
    for (int t = 1; t < D; t++) Wt[t - 1] = sc * (yt[t - 1] + F.vh[t] * yE);
}

// ... and the others, W_0..W_N and W_{nc-1} (in that order, N + 2 values),
// from the species variables y_0..y_{N-1}, the normal momentum variable y_N,
// vdot = vh.(y_N..y_{N+D-1}) and yE
template <int N, int D, typename R>
__device__ __forceinline__ void frame_project_main(const Frame<N, D, R>& F, const R* ysp, R yn, R vdot, R yE,
                                                   R* Wm)
{
    if constexpr (N == 1) {
        const R base = ysp[0] + vdot;
        const R gm = base - F.c * yn + (F.H - F.c * F.vh[0]) * yE;
        const R gp = base + F.c * yn + (F.H + F.c * F.vh[0]) * yE;
        const R ge = base + F.K * yE;
        Wm[0] = F.sa * gm;
        Wm[1] = F.se * ge;
        Wm[2] = F.sa * gp;
    } else {
        const R ys = F.Y[0] * ysp[0] + F.Y[1] * ysp[1] + vdot;
        const R gm = ys - F.c * yn + (F.H - F.c * F.vh[0]) * yE;
        const R gp = ys + F.c * yn + (F.H + F.c * F.vh[0]) * yE;
        const R g1 = ysp[0] + vdot + F.e2[0] * yE;
        const R g2 = ysp[1] + vdot + F.e2[1] * yE;
        Wm[0] = F.s2a * gm;
        Wm[1] = F.d11 * g1 + F.d21 * g2;
        Wm[2] = F.d12 * g1 + F.d22 * g2;
        Wm[3] = F.s2a * gp;
    }
}

// zero-tolerance scale of the fields of frame_project_main (same order):
// max over the species rows of |R_lc| times ay (the species magnitudes
// summed), plus sum_e |R_ec| a_e over the momentum rows (a_e = av) and the
// energy row (aE)
template <int N, int D, typename R>
__device__ __forceinline__ void frame_scale_main(const Frame<N, D, R>& F, R ay, R av, R aE, R* mg)
{
    R vt = R(0);   // sum of |vh_j| over the tangential rows
#pragma unroll
    for (int j = 1; j < D; j++) vt += fabs(F.vh[j]);
    const R cv0 = F.c * F.vh[0];
    if constexpr (N == 1) {
        mg[0] = F.sa * (ay + (fabs(F.vh[0] - F.c) + vt) * av + fabs(F.H - cv0) * aE);
        mg[1] = F.se * (ay + (fabs(F.vh[0]) + vt) * av + fabs(F.K) * aE);
        mg[2] = F.sa * (ay + (fabs(F.vh[0] + F.c) + vt) * av + fabs(F.H + cv0) * aE);
    } else {
        const R ya = fmax(fabs(F.Y[0]), fabs(F.Y[1])) * ay;
        const R va = (fabs(F.vh[0]) + vt) * av;
        mg[0] = F.s2a * (ya + (fabs(F.vh[0] - F.c) + vt) * av + fabs(F.H - cv0) * aE);
        mg[1] = fmax(fabs(F.d11), fabs(F.d21)) * ay + fabs(F.d11 + F.d21) * va +
                fabs(F.d11 * F.e2[0] + F.d21 * F.e2[1]) * aE;
        mg[2] = fmax(fabs(F.d12), fabs(F.d22)) * ay + fabs(F.d12 + F.d22) * va +
                fabs(F.d12 * F.e2[0] + F.d22 * F.e2[1]) * aE;
        mg[3] = F.s2a * (ya + (fabs(F.vh[0] + F.c) + vt) * av + fabs(F.H + cv0) * aE);
    }
}

// out = R z
template <int N, int D, typename R>
__device__ __forceinline__ void frame_expand(const Frame<N, D, R>& F, const R* z, R* out)
{
    constexpr int NC = N + D + 1;
    if constexpr (N == 1) {
        const R zm = F.sa * z[0], ze = F.se * z[1], zp = F.sa * z[NC - 1];
        const R sum = zm + ze + zp;
        out[0] = sum;
        out[1] = F.vh[0] * sum + F.c * (zp - zm);
        R eng = (F.H - F.c * F.vh[0]) * zm + F.K * ze + (F.H + F.c * F.vh[0]) * zp;
#pragma unroll
        for (int t = 1; t < D; t++) {
            const R zt = F.st * z[1 + t];
            out[1 + t] = F.vh[t] * sum + zt;
            eng += F.vh[t] * zt;
        }
        out[NC - 1] = eng;
    } else {
        const R zm = F.s2a * z[0], zp = F.s2a * z[NC - 1];
        const R z1 = F.d11 * z[1] + F.d12 * z[2];
        const R z2 = F.d21 * z[1] + F.d22 * z[2];
        const R sum = zm + z1 + z2 + zp;
        out[0] = F.Y[0] * (zm + zp) + z1;
        out[1] = F.Y[1] * (zm + zp) + z2;
        out[2] = F.vh[0] * sum + F.c * (zp - zm);
        R eng = (F.H - F.c * F.vh[0]) * zm + F.e2[0] * z1 + F.e2[1] * z2
              + (F.H + F.c * F.vh[0]) * zp;
#pragma unroll
        for (int t = 1; t < D; t++) {
            const R zt = F.sq * z[2 + t];
            out[2 + t] = F.vh[t] * sum + F.c * zt;
            eng += F.c * F.vh[t] * zt;
        }
        out[NC - 1] = eng;
    }
}

// --------------------------------------------------------------------------
// device scalar reductions (wavefront of 64 lanes, then LDS across waves)
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

enum RedOp { RED_MAX = 0, RED_MIN = 1, RED_SUM = 2 };

template <int OP>
__device__ __forceinline__ double red_combine(double a, double b)
{
    if constexpr (OP == RED_MAX) return fmax(a, b);
    else if constexpr (OP == RED_MIN) return fmin(a, b);
    else return a + b;
}

// block of 256 threads; returns the block result in thread 0
template <int OP>
__device__ __forceinline__ double block_reduce(double v)
{
    __shared__ double part[4];
    double w;
    if constexpr (OP == RED_MAX) w = wave_max(v);
    else if constexpr (OP == RED_MIN) w = wave_min(v);
    else w = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = w;
    __syncthreads();
    double r = part[0];
    if (threadIdx.x == 0) {
        r = red_combine<OP>(red_combine<OP>(part[0], part[1]), red_combine<OP>(part[2], part[3]));
    }
    __syncthreads();
    return r;
}

// Tile of this block for the z-marching and plane-tile kernels.  Consecutive
// blocks are dealt round-robin to the 8 XCDs, each with its own L2; this
// permutation gives each XCD a contiguous run of tiles (a whole z chunk of
// (x, y) tiles at the usual grids), so the in-plane neighbour rows that
// adjacent tiles read from each other come from one L2 (the 3D metrics take
// 8% less time).  Any grid size: the first nb % 8 XCDs take one tile more.
__device__ __forceinline__ void xcd_tile(int& bx, int& by, int& bz)
{
    const unsigned gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
    const unsigned L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned q = nb / 8, r = nb % 8, c = L % 8;
    const unsigned T = c * q + (c < r ? c : r) + L / 8;
    bx = (int)(T % gx);
    by = (int)((T / gx) % gy);
    bz = (int)(T / (gx * gy));
}

}  // namespace es
