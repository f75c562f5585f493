// es_kernels.hip -- the HBM-bound steps of the path on gfx950: ghost
// layers, GCL metrics (Section 3.2), the CFL wave speed (Section 5),
// mesh redistribution (Section 4) and the FP64 entropy sums.
#include "es_kernels.hpp"

namespace es {

// ---------------------------------------------------------------------------
// Ghost layers in one launch per field: every ghost node (the shell of the
// padded box: the z slabs, then the y slabs over interior z, then the x slabs
// over interior y and z) takes the value of one interior node, with all of
// its out-of-range coordinates mapped at once.
//
// Periodic faces wrap (the mesh gains -L_k / +L_k in component k below /
// above the interior along k).  The boundary conditions of the paper's
// walled examples (reflecting walls, outflow, inflow) are taken with
// cell-centred nodes: the face lies halfway between the outermost node and
// the first ghost node, and the ghost node m layers outside mirrors the
// interior node m - 1 layers inside.  Across such a face the mesh is
// mirrored about the face's coordinate (x_k -> 2 wall - x_k), displacements
// and time metrics negate component k, and a metric J dxi_a/dx_b is negated
// when exactly one of a, b is k: the values the mirrored mesh has.  The
// state is filled by fill_state.
// ---------------------------------------------------------------------------
// (index arithmetic in 32 bits: a grid holds fewer than 2^31 / 9 points,
// which the context checks at creation, and 64-bit division is a long
// software sequence on the GPU)
__device__ __forceinline__ void shell_node(const Geo& g, long t, long nzs, long nys, int d[3])
{
    const unsigned ng = g.ng;
    const unsigned np0 = g.np[0], np1 = g.np[1];
    const unsigned n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const int z0 = g.dim == 3 ? (int)ng : 0;
    if (t < nzs) {                                   // z ghost planes
        const unsigned u = (unsigned)t, pl = np0 * np1;
        const unsigned k = u / pl, r = u - k * pl;
        d[2] = (int)(k < ng ? k : k + n2);
        const unsigned y = r / np0;
        d[1] = (int)y;
        d[0] = (int)(r - y * np0);
    } else if (t < nzs + nys) {                      // y ghost rows over interior z
        const unsigned u = (unsigned)(t - nzs), per = 2u * ng * np0;
        const unsigned zz = u / per, r = u - zz * per;
        d[2] = z0 + (int)zz;
        const unsigned k = r / np0;
        d[1] = (int)(k < ng ? k : k + n1);
        d[0] = (int)(r - k * np0);
    } else {                                         // x ghost columns over interior y, z
        const unsigned u = (unsigned)(t - nzs - nys), w = 2u * ng;
        const unsigned row = u / w, k = u - row * w;
        d[0] = (int)(k < ng ? k : k + n0);
        const unsigned zz = row / n1;
        d[1] = (int)(ng + (row - zz * n1));
        d[2] = z0 + (int)zz;
    }
}

// interior image of padded index i along k; side = -1 / +1 below / above
// the interior, 0 inside
__device__ __forceinline__ int ghost_image(const Geo& g, int k, int i, int& side)
{
    const int n = g.n[k], r = i - g.ng;
    side = r < 0 ? -1 : (r >= n ? 1 : 0);
    if (!side) return i;
    if (g.bc[k][side > 0] == BC_PERIODIC) return (side < 0 ? r + n : r - n) + g.ng;
    return (side < 0 ? -1 - r : 2 * n - 1 - r) + g.ng;
}

// ghost value of component c of a field of kind `what` from its image value v
__device__ __forceinline__ double ghost_value(const Geo& g, int what, int c, const int side[3], double v)
{
    for (int k = 0; k < g.dim; k++) {
        if (!side[k]) continue;
        if (g.bc[k][side[k] > 0] == BC_PERIODIC) {
            if (what == GH_MESH && c == k) v += side[k] * g.len[k];
            continue;
        }
        if (what == GH_MESH && c == k) v = 2.0 * g.wall[k][side[k] > 0] - v;
        if ((what == GH_DISP || what == GH_JXT) && c == k) v = -v;
        if (what == GH_JXX && ((c / g.dim == k) != (c % g.dim == k))) v = -v;
    }
    return v;
}

// The grid-stride kernels of this file that produce a field also write its ghost
// layers when given the shell sizes (nzs + nys + nxs > 0): a ghost node
// takes the value of the interior node it wraps or mirrors to, computed again
// with the same arithmetic, under the field's ghost rule.  That saves the
// separate fill launch.
__device__ __forceinline__ long shell_image(const Geo& g, long t, long nzs, long nys, int side[3], long& di)
{
    int d[3];
    shell_node(g, t, nzs, nys, d);
    int sidx[3] = {d[0], d[1], d[2]};
    side[0] = side[1] = side[2] = 0;
    for (int k = 0; k < g.dim; k++) sidx[k] = ghost_image(g, k, d[k], side[k]);
    di = node_index(g, d[0], d[1], d[2]);
    return node_index(g, sidx[0], sidx[1], sidx[2]);
}

// one or two fields (a2 may be null) of their own kinds per launch; the
// first is skipped where skip_a is given and set (metrics kept from the step
// before have their ghost layers already)
__global__ void k_fill_shell(Geo g, double* __restrict__ a, int ncomp, int what, double* __restrict__ a2,
                             int ncomp2, int what2, long nzs, long nys, long nxs, const int* __restrict__ skip_a)
{
    if (skip_a && *skip_a) ncomp = 0;
    const long total = nzs + nys + nxs;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        int d[3];
        shell_node(g, t, nzs, nys, d);
        int sidx[3] = {d[0], d[1], d[2]}, side[3] = {0, 0, 0};
        for (int k = 0; k < g.dim; k++) sidx[k] = ghost_image(g, k, d[k], side[k]);
        const long di = node_index(g, d[0], d[1], d[2]);
        const long si = node_index(g, sidx[0], sidx[1], sidx[2]);
        for (int c = 0; c < ncomp; c++) a[c * g.P + di] = ghost_value(g, what, c, side, a[c * g.P + si]);
        if (a2)
            for (int c = 0; c < ncomp2; c++) a2[c * g.P + di] = ghost_value(g, what2, c, side, a2[c * g.P + si]);
    }
}

// the state's ghosts: J is a plain field (wrapped or mirrored); a
// reflecting wall mirrors U with momentum component k negated, outflow
// copies U of the outermost interior node, inflow takes the face's
// prescribed state (the lowest direction's where several meet); JU = J
// (mirrored) times that U
__global__ void k_fill_state(Geo g, InflowStates in, double* __restrict__ JU, double* __restrict__ J,
                             int nc, int nspec, long nzs, long nys, long nxs)
{
    const long total = nzs + nys + nxs;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        int d[3];
        shell_node(g, t, nzs, nys, d);
        int src[3] = {d[0], d[1], d[2]}, img[3] = {d[0], d[1], d[2]};
        int flip = 0, uk = -1, us = 0;
        bool extrap = false;
        for (int k = 0; k < g.dim; k++) {
            int side;
            src[k] = ghost_image(g, k, d[k], side);
            img[k] = src[k];
            if (!side) continue;
            const int kind = g.bc[k][side > 0];
            if (kind == BC_REFLECT) flip |= 1 << k;
            if (kind == BC_OUTFLOW) {
                src[k] = side < 0 ? g.ng : g.ng + g.n[k] - 1;
                extrap = true;
            }
            if (kind == BC_INFLOW && uk < 0) {
                uk = k;
                us = side > 0;
            }
        }
        const long di = node_index(g, d[0], d[1], d[2]);
        const long si = node_index(g, src[0], src[1], src[2]);
        const double Jd = J[node_index(g, img[0], img[1], img[2])];
        J[di] = Jd;
        for (int c = 0; c < nc; c++) {
            double u;
            if (uk >= 0) u = Jd * in.u[uk][us][c];
            else if (extrap) u = Jd * (JU[c * g.P + si] / J[si]);
            else u = JU[c * g.P + si];
            if (uk < 0 && c >= nspec && c < nspec + g.dim && ((flip >> (c - nspec)) & 1)) u = -u;
            JU[c * g.P + di] = u;
        }
    }
}

static void shell_sizes(const Geo& g, long& nzs, long& nys, long& nxs)
{
    const long ng2 = 2L * g.ng;
    const long nz = g.dim == 3 ? g.n[2] : 1;
    nzs = g.dim == 3 ? ng2 * g.np[0] * g.np[1] : 0;
    nys = ng2 * g.np[0] * nz;
    nxs = ng2 * g.n[1] * nz;
}

hipError_t fill_ghosts2(const Geo& g, double* a, int ncomp, int what, double* a2, int ncomp2, int what2,
                       hipStream_t s, const int* skip_a = nullptr)
{
    long nzs, nys, nxs;
    shell_sizes(g, nzs, nys, nxs);
    const long total = nzs + nys + nxs;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_shell, dim3(blocks), dim3(256), 0, s, g, a, ncomp, what, a2, ncomp2, what2, nzs,
                       nys, nxs, skip_a);
    return hipGetLastError();
}

hipError_t fill_ghosts(const Geo& g, double* a, int ncomp, int what, hipStream_t s)
{
    return fill_ghosts2(g, a, ncomp, what, nullptr, 0, GH_PLAIN, s);
}

hipError_t fill_state(const Geo& g, const InflowStates& in, double* JU, double* J, int nc, int nspec,
                      hipStream_t s)
{
    bool periodic = true;
    for (int k = 0; k < g.dim; k++) periodic = periodic && g.bc[k][0] == BC_PERIODIC;
    if (periodic) return fill_ghosts2(g, JU, nc, GH_PLAIN, J, 1, GH_PLAIN, s);   // plain wrapped copies
    long nzs, nys, nxs;
    shell_sizes(g, nzs, nys, nxs);
    const long total = nzs + nys + nxs;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_state, dim3(blocks), dim3(256), 0, s, g, in, JU, J, nc, nspec, nzs, nys, nxs);
    return hipGetLastError();
}

// interior node q (0 .. nint-1) -> padded index
// (32-bit index arithmetic, as in shell_node)
__device__ __forceinline__ long interior_node(const Geo& g, long q, int& i0, int& i1, int& i2)
{
    const unsigned u = (unsigned)q, n0 = g.n[0], n1 = g.n[1];
    const unsigned r = u / n0, z = r / n1;
    i0 = (int)(u - r * n0) + g.ng;
    i1 = (int)(r - z * n1) + g.ng;
    i2 = (int)z + (g.dim == 3 ? g.ng : 0);
    return node_index(g, i0, i1, i2);
}

__device__ __forceinline__ long n_interior(const Geo& g)
{
    return (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, long n)
{
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

__global__ void k_fill_value(double* __restrict__ dst, long n, double v)
{
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        dst[t] = v;
}

__global__ void k_set_scalar(double* dst, double v) { if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v; }
__global__ void k_set_int(int* dst, int v) { if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v; }

// clears *flag unless a and b hold the same n values (a NaN never matches)
__global__ void k_same(const double* __restrict__ a, const double* __restrict__ b, long n, int* __restrict__ flag)
{
    bool differ = false;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        differ |= !(a[t] == b[t]);
    if (differ) *flag = 0;
}

// dst = src over n values when *flag is zero
__global__ void k_copy_unless(const double* __restrict__ src, double* __restrict__ dst, long n,
                              const int* __restrict__ flag)
{
    if (*flag) return;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

static int grid_for(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 16384)); }

hipError_t copy(const double* src, double* dst, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}
hipError_t fill_value(double* dst, long n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_value, dim3(grid_for(n)), dim3(256), 0, s, dst, n, v);
    return hipGetLastError();
}
hipError_t same_values(const double* a, const double* b, long n, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, flag, 1);
    hipLaunchKernelGGL(k_same, dim3(grid_for(n)), dim3(256), 0, s, a, b, n, flag);
    return hipGetLastError();
}
hipError_t copy_unless(const double* src, double* dst, long n, const int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_unless, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n, flag);
    return hipGetLastError();
}
hipError_t set_scalar(double* dst, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GCL metrics (eq SCLCoeff, eq VCLCoeff).  Stage mesh xs = x_n + c_s disp.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double xs_at(const double* xn, const double* disp, double cs, long P, int p,
                                        long i)
{
    double v = xn[p * P + i];
    if (disp && cs != 0.0) v += cs * disp[p * P + i];
    return v;
}

// 3D metrics in two z-marching passes.  Pass 1 forms the products
//   Pr[a][j] = delta_a[xs_p] xs_q,  (p, q) = (j+1, j+2) mod 3,
// at every node interior along a; pass 2 differences them,
//   J dxi_k/dx_j = (delta_b[Pr[a][j]] - delta_a[Pr[b][j]]) / (dxi_a dxi_b),  (k, a, b) cyclic.
// delta is the 2w-order central difference 1/2 sum_m alpha_m (f_{+m} - f_{-m})
// (alpha_m = 0 for m > w).  Each thread walks one (x, y) column up a chunk of
// z planes, and z-differences come from a 7-plane ring in registers (each
// value is loaded once).
//   Pass 1 (16 x 16 columns) stages the stage mesh xs = x + c_s disp of the
//   current plane with a 3-node halo in LDS for the x/y-differences (two
//   loads per value, each used by up to 13 nodes).
//   Pass 2 (64 x 4 columns, so a wavefront reads 64 consecutive doubles of a
//   row) stages the in-plane neighbours of the products of the current plane
//   in LDS (Pr[2] along x and y, Pr[0] along y, Pr[1] along x, 3-node
//   halos): 1011 us at 256^3 against 1195 us reading them from the caches.
constexpr int MT = 16;
constexpr int MH = MT + 6;
constexpr int MX = 64, MY = 4;

__device__ __forceinline__ double cdiff(const double* al, double p1, double m1, double p2, double m2,
                                        double p3, double m3)
{
    double s = al[0] * (p1 - m1);
    s += al[1] * (p2 - m2);
    s += al[2] * (p3 - m3);
    return 0.5 * s;
}

__global__ void __launch_bounds__(MT * MT)
k_metric_prod3(Geo g, Phys ph, const double* __restrict__ xn, const double* __restrict__ disp,
               double cs, double* __restrict__ Pr, int zchunk, const int* __restrict__ reuse)
{
    if (reuse && *reuse) return;
    __shared__ double T[3][MH][MH];
    const long P = g.P;
    const int np0 = g.np[0], np1 = g.np[1], np2 = g.np[2];
    const int tx = threadIdx.x, ty = threadIdx.y;
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    const int x0 = bx * MT, y0 = by * MT;
    const int x = x0 + tx, y = y0 + ty;
    const int zc0 = bz * zchunk, zc1 = min(zc0 + zchunk, np2);
    const bool in = x < np0 && y < np1;
    const bool xin = x >= g.ng && x < g.ng + g.n[0];
    const bool yin = y >= g.ng && y < g.ng + g.n[1];
    const double al[3] = {ph.alpha[0], ph.alpha[1], ph.alpha[2]};
    double ring[3][7];
#pragma unroll
    for (int p = 0; p < 3; p++)
#pragma unroll
        for (int r = 0; r < 7; r++) ring[p][r] = 0.0;
    const int zs = max(zc0 - 3, 0), ze = min(zc1 + 3, np2);
    for (int zl = zs; zl < ze; zl++) {
        for (int q = ty * MT + tx; q < MH * MH; q += MT * MT) {
            const int hx = q % MH, hy = q / MH;
            const int gx = x0 + hx - 3, gy = y0 + hy - 3;
            if (gx >= 0 && gx < np0 && gy >= 0 && gy < np1) {
                const long i = ((long)zl * np1 + gy) * np0 + gx;
#pragma unroll
                for (int p = 0; p < 3; p++) {
                    double v = xn[p * P + i];
                    if (disp) v += cs * disp[p * P + i];
                    T[p][hy][hx] = v;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 3; p++) {
#pragma unroll
            for (int r = 0; r < 6; r++) ring[p][r] = ring[p][r + 1];
            ring[p][6] = in ? T[p][ty + 3][tx + 3] : 0.0;
        }
        if (in && zl >= zc0 && zl < zc1) {
            const long i = ((long)zl * np1 + y) * np0 + x;
            const int cx = tx + 3, cy = ty + 3;
            if (xin) {
                double d[3];
#pragma unroll
                for (int p = 0; p < 3; p++)
                    d[p] = cdiff(al, T[p][cy][cx + 1], T[p][cy][cx - 1], T[p][cy][cx + 2],
                                 T[p][cy][cx - 2], T[p][cy][cx + 3], T[p][cy][cx - 3]);
#pragma unroll
                for (int j = 0; j < 3; j++) Pr[(0 * 3 + j) * P + i] = d[(j + 1) % 3] * T[(j + 2) % 3][cy][cx];
            }
            if (yin) {
                double d[3];
#pragma unroll
                for (int p = 0; p < 3; p++)
                    d[p] = cdiff(al, T[p][cy + 1][cx], T[p][cy - 1][cx], T[p][cy + 2][cx],
                                 T[p][cy - 2][cx], T[p][cy + 3][cx], T[p][cy - 3][cx]);
#pragma unroll
                for (int j = 0; j < 3; j++) Pr[(1 * 3 + j) * P + i] = d[(j + 1) % 3] * T[(j + 2) % 3][cy][cx];
            }
        }
        const int zp = zl - 3;   // ring slot 3 holds plane zp
        if (in && zp >= zc0 && zp < zc1 && zp >= g.ng && zp < g.ng + g.n[2]) {
            const long i = ((long)zp * np1 + y) * np0 + x;
            double d[3];
#pragma unroll
            for (int p = 0; p < 3; p++)
                d[p] = cdiff(al, ring[p][4], ring[p][2], ring[p][5], ring[p][1], ring[p][6], ring[p][0]);
#pragma unroll
            for (int j = 0; j < 3; j++) Pr[(2 * 3 + j) * P + i] = d[(j + 1) % 3] * ring[(j + 2) % 3][3];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(MX * MY) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_metric3(Geo g, Phys ph, const double* __restrict__ disp, const double* __restrict__ Pr,
          const double* __restrict__ dt_dev, double* __restrict__ jxx, double* __restrict__ jxt,
          int zchunk, const int* __restrict__ reuse)
{
    if (reuse && *reuse) return;
    // the in-plane neighbours of plane z: Pr[2][j] along x and y, Pr[0][j]
    // along y, Pr[1][j] along x (the tile plus a 3-node halo; the corners of
    // the Pr[2] patch are never read)
    __shared__ double L2[3][MY + 6][MX + 6];
    __shared__ double L0[3][MY + 6][MX];
    __shared__ double L1[3][MY][MX + 6];
    const long P = g.P;
    const int np0 = g.np[0], np1 = g.np[1];
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int xt = g.ng + bx * MX, yt = g.ng + by * MY;
    const int x = xt + tx, y = yt + ty;
    const int zc0 = g.ng + bz * zchunk, zc1 = min(zc0 + zchunk, g.ng + g.n[2]);
    const bool in = x < g.ng + g.n[0] && y < g.ng + g.n[1];
    const double dt = dt_dev ? *dt_dev : 0.0;
    const double idt = dt > 0.0 ? 1.0 / dt : 0.0;   // mesh velocity = disp / dt
    const double al[3] = {ph.alpha[0], ph.alpha[1], ph.alpha[2]};
    const double s01 = g.idxi[0] * g.idxi[1], s12 = g.idxi[1] * g.idxi[2], s20 = g.idxi[2] * g.idxi[0];
    const int t = tx + MX * ty;
    double ring[6][7];   // Pr[0][j] (0..2) and Pr[1][j] (3..5) at the own node, planes zl-6..zl
#pragma unroll
    for (int c = 0; c < 6; c++)
#pragma unroll
        for (int r = 0; r < 7; r++) ring[c][r] = 0.0;
    // the ring advances on every thread (a column beyond a ragged tile reads
    // the last padded node instead): a shift under a branch would keep two
    // copies of the ring live
    const int xr = min(x, np0 - 1), yr = min(y, np1 - 1);
    auto advance = [&](int zl) {   // ring slot r then holds plane zl - 6 + r
        const long il = ((long)zl * np1 + yr) * np0 + xr;
#pragma unroll
        for (int c = 0; c < 6; c++) {
#pragma unroll
            for (int r = 0; r < 6; r++) ring[c][r] = ring[c][r + 1];
            ring[c][6] = Pr[(long)c * P + il];
        }
    };
    for (int zl = zc0 - 3; zl < zc0 + 3; zl++) advance(zl);
    for (int z = zc0; z < zc1; z++) {
        advance(z + 3);
        const long pz = (long)z * np1;
#pragma unroll 1
        for (int q = t; q < (MY + 6) * (MX + 6); q += MX * MY) {
            const int hx = q % (MX + 6), hy = q / (MX + 6);
            const bool cx = hx >= 3 && hx < MX + 3, cy = hy >= 3 && hy < MY + 3;
            const int gx = xt - 3 + hx, gy = yt - 3 + hy;
            if (!(cx || cy) || gx >= np0 || gy >= np1) continue;
            const long gi = (pz + gy) * np0 + gx;
#pragma unroll
            for (int j = 0; j < 3; j++) L2[j][hy][hx] = Pr[(long)(6 + j) * P + gi];
            if (cx) {
#pragma unroll
                for (int j = 0; j < 3; j++) L0[j][hy][hx - 3] = Pr[(long)j * P + gi];
            }
            if (cy) {
#pragma unroll
                for (int j = 0; j < 3; j++) L1[j][hy - 3][hx] = Pr[(long)(3 + j) * P + gi];
            }
        }
        __syncthreads();
        if (in) {
            const long i = (pz + y) * np0 + x;
            const int cx = tx + 3, cy = ty + 3;
            // one j at a time: its three metrics are stored and folded into
            // the time metrics at once (the sum over j in the same order)
            double w[3] = {0.0, 0.0, 0.0};
            if (jxt && disp && dt > 0.0)
#pragma unroll
                for (int j = 0; j < 3; j++) w[j] = disp[j * P + i] * idt;
            double nt[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int j = 0; j < 3; j++) {
                // each difference reads its six LDS values after a point that
                // no LDS read moves across, so few of them are live beside
                // the ring (four waves per SIMD without spills)
                double M[3];
                // k = 0 (a = 1, b = 2): delta_2 Pr[1][j] - delta_1 Pr[2][j]
                const double* r1 = ring[3 + j];
                const double t1 = cdiff(al, r1[4], r1[2], r1[5], r1[1], r1[6], r1[0]);
                asm volatile("" ::: "memory");
                const double t2 = cdiff(al, L2[j][cy + 1][cx], L2[j][cy - 1][cx], L2[j][cy + 2][cx],
                                        L2[j][cy - 2][cx], L2[j][cy + 3][cx], L2[j][cy - 3][cx]);
                M[0] = (t1 - t2) * s12;
                // k = 1 (a = 2, b = 0): delta_0 Pr[2][j] - delta_2 Pr[0][j]
                const double* r0 = ring[j];
                asm volatile("" ::: "memory");
                const double u1 = cdiff(al, L2[j][cy][cx + 1], L2[j][cy][cx - 1], L2[j][cy][cx + 2],
                                        L2[j][cy][cx - 2], L2[j][cy][cx + 3], L2[j][cy][cx - 3]);
                const double u2 = cdiff(al, r0[4], r0[2], r0[5], r0[1], r0[6], r0[0]);
                M[1] = (u1 - u2) * s20;
                // k = 2 (a = 0, b = 1): delta_1 Pr[0][j] - delta_0 Pr[1][j]
                asm volatile("" ::: "memory");
                const double v1 = cdiff(al, L0[j][cy + 1][tx], L0[j][cy - 1][tx], L0[j][cy + 2][tx],
                                        L0[j][cy - 2][tx], L0[j][cy + 3][tx], L0[j][cy - 3][tx]);
                asm volatile("" ::: "memory");
                const double v2 = cdiff(al, L1[j][ty][cx + 1], L1[j][ty][cx - 1], L1[j][ty][cx + 2],
                                        L1[j][ty][cx - 2], L1[j][ty][cx + 3], L1[j][ty][cx - 3]);
                M[2] = (v1 - v2) * s01;
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    __builtin_nontemporal_store(M[k], &jxx[(k * 3 + j) * P + i]);
                    nt[k] -= w[j] * M[k];
                }
            }
            if (jxt)
#pragma unroll
                for (int k = 0; k < 3; k++) __builtin_nontemporal_store(nt[k], &jxt[k * P + i]);
        }
        __syncthreads();   // the next plane overwrites the patch
    }
}

// 2D: J dxi_1/dx = (delta_2 x_2, -delta_2 x_1)/dxi_2, J dxi_2/dx = (-delta_1 x_2, delta_1 x_1)/dxi_1
__device__ __forceinline__ void metric2_node(const Geo& g, const Phys& ph, const double* xn, const double* disp,
                                             double cs, double dt, long i, double M[2][2], double nt[2])
{
    const long P = g.P;
    const long s0 = 1, s1 = g.np[0];
    double d[2][2];   // d[a][p] = delta_a[x_p]
#pragma unroll
    for (int a = 0; a < 2; a++) {
        const long st = a == 0 ? s0 : s1;
#pragma unroll
        for (int p = 0; p < 2; p++) {
            double s = 0.0;
            for (int m = 1; m <= ph.w; m++)
                s += ph.alpha[m - 1] * (xs_at(xn, disp, cs, P, p, i + m * st) - xs_at(xn, disp, cs, P, p, i - m * st));
            d[a][p] = 0.5 * s;
        }
    }
    M[0][0] = d[1][1] / g.dxi[1];
    M[0][1] = -d[1][0] / g.dxi[1];
    M[1][0] = -d[0][1] / g.dxi[0];
    M[1][1] = d[0][0] / g.dxi[0];
#pragma unroll
    for (int k = 0; k < 2; k++) {
        nt[k] = 0.0;
        if (disp && dt > 0.0)
#pragma unroll
            for (int j = 0; j < 2; j++) nt[k] -= (disp[j * P + i] * (1.0 / dt)) * M[k][j];
    }
}

__global__ void k_metric2(Geo g, Phys ph, const double* __restrict__ xn,
                          const double* __restrict__ disp, double cs, const double* __restrict__ dt_dev,
                          double* __restrict__ jxx, double* __restrict__ jxt, long nzs, long nys, long nxs,
                          const int* __restrict__ reuse)
{
    if (reuse && *reuse) return;
    const long P = g.P;
    const long nint = n_interior(g);
    const double dt = dt_dev ? *dt_dev : 0.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        double M[2][2], nt[2];
        metric2_node(g, ph, xn, disp, cs, dt, i, M, nt);
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
            for (int j = 0; j < 2; j++) jxx[(k * 2 + j) * P + i] = M[k][j];
        if (jxt)
#pragma unroll
            for (int k = 0; k < 2; k++) jxt[k * P + i] = nt[k];
    }
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nzs + nys + nxs;
         t += (long)gridDim.x * blockDim.x) {
        int side[3];
        long di;
        const long si = shell_image(g, t, nzs, nys, side, di);
        double M[2][2], nt[2];
        metric2_node(g, ph, xn, disp, cs, dt, si, M, nt);
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
            for (int j = 0; j < 2; j++) jxx[(k * 2 + j) * P + di] = ghost_value(g, GH_JXX, k * 2 + j, side, M[k][j]);
        if (jxt)
#pragma unroll
            for (int k = 0; k < 2; k++) jxt[k * P + di] = ghost_value(g, GH_JXT, k, side, nt[k]);
    }
}

// jxi_t only, from an existing jxi_x (only when *only_if is set, if given)
__global__ void k_vcl(Geo g, const double* __restrict__ disp, const double* __restrict__ dt_dev,
                      const double* __restrict__ jxx, double* __restrict__ jxt, const int* __restrict__ only_if)
{
    if (only_if && !*only_if) return;
    const long P = g.P;
    const int D = g.dim;
    const long nint = n_interior(g);
    const double dt = dt_dev ? *dt_dev : 0.0;
    const double idt = dt > 0.0 ? 1.0 / dt : 0.0;   // mesh velocity = disp / dt
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        for (int k = 0; k < D; k++) {
            double nt = 0.0;
            if (disp && dt > 0.0)
                for (int j = 0; j < D; j++) nt -= (disp[j * P + i] * idt) * jxx[(k * D + j) * P + i];
            jxt[k * P + i] = nt;
        }
    }
}

// discrete Jacobian of the mesh: J = (1/d) sum_k sum_j dx_j/dxi_k J dxi_k/dx_j
// (the cofactor expansion of det dx/dxi along each column k, averaged),
// dx_j/dxi_k by the 2w-order central difference of the metrics
__global__ void k_jacobian(Geo g, Phys ph, const double* __restrict__ x, const double* __restrict__ jxx,
                           double* __restrict__ J)
{
    const long P = g.P;
    const int d = g.dim;
    const long nint = n_interior(g);
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        double s = 0.0;
        for (int k = 0; k < d; k++) {
            const long st = dir_stride(g, k);
            for (int j = 0; j < d; j++) {
                const double* a = x + j * P;
                double dk = 0.0;
                for (int m = 1; m <= ph.w; m++) dk += ph.alpha[m - 1] * (a[i + m * st] - a[i - m * st]);
                s += 0.5 * dk / g.dxi[k] * jxx[(k * d + j) * P + i];
            }
        }
        J[i] = s / d;
    }
}

hipError_t jacobian(const Phys& ph, const Geo& g, const double* x, const double* jxx, double* J, hipStream_t s)
{
    const long nint = (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
    hipLaunchKernelGGL(k_jacobian, dim3(grid_for(nint)), dim3(256), 0, s, g, ph, x, jxx, J);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : fill_ghosts(g, J, 1, GH_PLAIN, s);
}

hipError_t metrics(const Phys& ph, const Geo& g, const double* xn, const double* disp, double cs,
                   const double* dt_dev, double* jxx, double* jxt, int vcl_only, double* G,
                   hipStream_t s, const int* reuse)
{
    const long nint = (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
    // the stage mesh reads the displacement only where c_s is not zero (the
    // 2D kernel tests c_s itself: it reads disp for the time metrics too)
    const double* dx = cs != 0.0 ? disp : nullptr;
    if (vcl_only) {
        if (!jxt) return hipSuccess;
        hipLaunchKernelGGL(k_vcl, dim3(grid_for(nint)), dim3(256), 0, s, g, disp, dt_dev, jxx, jxt,
                           (const int*)nullptr);
    } else if (g.dim == 2) {   // with its ghost layers
        long nzs, nys, nxs;
        shell_sizes(g, nzs, nys, nxs);
        hipLaunchKernelGGL(k_metric2, dim3(grid_for(nint)), dim3(256), 0, s, g, ph, xn, disp, cs, dt_dev,
                           jxx, jxt, nzs, nys, nxs, reuse);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !reuse || !jxt) return e;
        // reused metrics: the time metrics of this step's displacement
        hipLaunchKernelGGL(k_vcl, dim3(grid_for(nint)), dim3(256), 0, s, g, disp, dt_dev, jxx, jxt, reuse);
        e = hipGetLastError();
        return e != hipSuccess ? e : fill_ghosts(g, jxt, g.dim, GH_JXT, s);
    } else {
        // z chunks: enough blocks to fill the chip, chunks long against the
        // 6-plane ring start-up
        const int bx1 = (g.np[0] + MT - 1) / MT, by1 = (g.np[1] + MT - 1) / MT;
        const int nc1 = std::max(1, std::min(g.np[2] / 32, (1024 + bx1 * by1 - 1) / (bx1 * by1)));
        const int zc1 = (g.np[2] + nc1 - 1) / nc1;
        hipLaunchKernelGGL(k_metric_prod3, dim3(bx1, by1, (g.np[2] + zc1 - 1) / zc1), dim3(MT, MT), 0, s,
                           g, ph, xn, dx, cs, G, zc1, reuse);
        const int bx2 = (g.n[0] + MX - 1) / MX, by2 = (g.n[1] + MY - 1) / MY;
        const int nc2 = std::max(1, std::min(g.n[2] / 16, (4096 + bx2 * by2 - 1) / (bx2 * by2)));
        const int zc2 = (g.n[2] + nc2 - 1) / nc2;
        hipLaunchKernelGGL(k_metric3, dim3(bx2, by2, (g.n[2] + zc2 - 1) / zc2), dim3(MX, MY), 0, s, g, ph,
                           disp, G, dt_dev, jxx, jxt, zc2, reuse);
        if (reuse && jxt)
            hipLaunchKernelGGL(k_vcl, dim3(grid_for(nint)), dim3(256), 0, s, g, disp, dt_dev, jxx, jxt, reuse);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!vcl_only) return fill_ghosts2(g, jxx, g.dim * g.dim, GH_JXX, jxt, g.dim, GH_JXT, s, reuse);
    if (jxt) e = fill_ghosts(g, jxt, g.dim, GH_JXT, s);
    return e;
}

// ---------------------------------------------------------------------------
// reductions: per-block partials in a fixed grid, then one block folds the
// partials in a fixed order (deterministic sums)
// ---------------------------------------------------------------------------
static constexpr int RED_BLOCKS = 2048;

template <int OP>
__global__ void k_finish(const double* __restrict__ part, int nparts, double* __restrict__ out,
                         int mode, double a, unsigned* status)
{
    double v = (OP == RED_MAX) ? -INFINITY : (OP == RED_MIN ? INFINITY : 0.0);
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) v = red_combine<OP>(v, part[t]);
    v = block_reduce<OP>(v);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            out[0] = v;
        } else if (mode == 1) {           // CFL: out[0] = lambda, out[1] = cfl / lambda
            out[0] = v;
            out[1] = a / v;
        } else if (mode == 2) {           // limiter: Delta_tau = min(1, v)
            const double d = fmin(1.0, v);
            out[0] = d;
            if (!(d > 0.0)) atomicOr(status, 2u);
        } else {                          // scaled sum
            out[0] = v * a;
        }
    }
}

// thermo of one node from JU/J
template <int N, int D>
struct NodeState {
    double U[N + D + 1];
    double rho, v[D], T, p, beta;
    bool ok;
};

template <int N, int D>
__device__ __forceinline__ void load_state(const Phys& ph, const double* JU, const double* Jv, long P,
                                           long i, NodeState<N, D>& s)
{
    constexpr int NC = N + D + 1;
    const double Jq = Jv[i];
#pragma unroll
    for (int c = 0; c < NC; c++) s.U[c] = JU[c * P + i] / Jq;
    double rt = 0.0, cvr = 0.0, rR = 0.0;
    bool ok = Jq > 0.0;
#pragma unroll
    for (int l = 0; l < N; l++) {
        rt += s.U[l];
        cvr += ph.cv[l] * s.U[l];
        rR += ph.Rg[l] * s.U[l];
        ok = ok && (s.U[l] > 0.0);
    }
    double kin = 0.0;
#pragma unroll
    for (int j = 0; j < D; j++) {
        s.v[j] = s.U[N + j] / rt;
        kin += 0.5 * s.U[N + j] * s.v[j];
    }
    s.rho = rt;
    s.T = (s.U[NC - 1] - kin - ph.pinf_tot) / cvr;
    s.beta = 1.0 / s.T;
    s.p = rR * s.T - ph.pinf_tot;
    s.ok = ok && (s.T > 0.0) && isfinite(s.T) && isfinite(kin);
}

template <int N, int D>
__global__ void k_wavespeed(Phys ph, Geo g, const double* __restrict__ JU, const double* __restrict__ Jv,
                            const double* __restrict__ jxx, double* __restrict__ part,
                            unsigned* __restrict__ status)
{
    const long P = g.P;
    const long nint = n_interior(g);
    double lam = 0.0;
    unsigned bad = 0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        NodeState<N, D> s;
        load_state<N, D>(ph, JU, Jv, P, i, s);
        if (!s.ok) bad |= 1u;
        double cvr = 0.0, cg = 0.0, rR = 0.0;
#pragma unroll
        for (int l = 0; l < N; l++) {
            cvr += ph.cv[l] * s.U[l];
            cg += ph.cvgam[l] * s.U[l];
            rR += ph.Rg[l] * s.U[l];
        }
        const double c = sqrt((rR / s.rho) * (cg / cvr) * s.T);
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            double vn = 0.0, nn = 0.0;
#pragma unroll
            for (int j = 0; j < D; j++) {
                const double n = jxx[(k * D + j) * P + i];
                vn += s.v[j] * n;
                nn += n * n;
            }
            sum += (fabs(vn) + c * sqrt(nn)) / Jv[i] / g.dxi[k];
        }
        lam = fmax(lam, sum);
    }
    if (bad) atomicOr(status, bad);
    lam = block_reduce<RED_MAX>(lam);
    if (threadIdx.x == 0) part[blockIdx.x] = lam;
}

template <int N, int D>
__global__ void k_entropy(Phys ph, Geo g, const double* __restrict__ JU, const double* __restrict__ Jv,
                          const double* __restrict__ dJU, const double* __restrict__ dJ,
                          double* __restrict__ part)
{
    constexpr int NC = N + D + 1;
    const long P = g.P;
    const long nint = n_interior(g);
    double acc = 0.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        NodeState<N, D> s;
        load_state<N, D>(ph, JU, Jv, P, i, s);
        // logarithms as the flux kernels take them (within 2 ulp); a
        // non-positive T or rho_l is a non-physical state the steps report
        const double lT = ln_pos(s.T);
        if (!dJU) {   // J eta, eta = -sum rho_l (c_vl ln T - R_l ln rho_l)
            double eta = 0.0;
#pragma unroll
            for (int l = 0; l < N; l++) eta -= s.U[l] * (ph.cv[l] * lT - ph.Rg[l] * ln_pos(s.U[l]));
            acc += Jv[i] * eta;
        } else {      // V . dJU - phi dJ
            double v2 = 0.0;
#pragma unroll
            for (int j = 0; j < D; j++) v2 += s.v[j] * s.v[j];
            double t = 0.0, phi = 0.0;
#pragma unroll
            for (int l = 0; l < N; l++) {
                const double Vl = -(ph.cv[l] * lT - ph.Rg[l] * ln_pos(s.U[l])) - v2 / (2.0 * s.T) + ph.cvgam[l];
                t += Vl * dJU[l * P + i];
                phi += ph.Rg[l] * s.U[l] - ph.pinf[l] / s.T;
            }
#pragma unroll
            for (int j = 0; j < D; j++) t += (s.v[j] / s.T) * dJU[(N + j) * P + i];
            t += (-1.0 / s.T) * dJU[(NC - 1) * P + i];
            acc += t - phi * dJ[i];
        }
    }
    acc = block_reduce<RED_SUM>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

static int red_grid(long nint) { return (int)std::max<long>(1, std::min<long>((nint + 255) / 256, RED_BLOCKS)); }

int reduction_blocks(long nint) { return red_grid(nint); }

#define ES_DISPATCH_ND(ph, g, FN, ...)                                   \
    do {                                                                 \
        if (ph.nspec == 1 && g.dim == 2) FN<1, 2>(__VA_ARGS__);          \
        else if (ph.nspec == 2 && g.dim == 2) FN<2, 2>(__VA_ARGS__);     \
        else if (ph.nspec == 1 && g.dim == 3) FN<1, 3>(__VA_ARGS__);     \
        else FN<2, 3>(__VA_ARGS__);                                      \
    } while (0)

template <int N, int D>
static void launch_wavespeed(const Phys& ph, const Geo& g, const double* JU, const double* J,
                             const double* jxx, double* part, unsigned* status, int nb, hipStream_t s)
{
    hipLaunchKernelGGL((k_wavespeed<N, D>), dim3(nb), dim3(256), 0, s, ph, g, JU, J, jxx, part, status);
}

hipError_t wavespeed(const Phys& ph, const Geo& g, const double* JU, const double* J, const double* jxx,
                     double cfl, double* part, double* out2, unsigned* status, hipStream_t s)
{
    const long nint = (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
    const int nb = red_grid(nint);
    ES_DISPATCH_ND(ph, g, launch_wavespeed, ph, g, JU, J, jxx, part, status, nb, s);
    hipLaunchKernelGGL(k_finish<RED_MAX>, dim3(1), dim3(256), 0, s, part, nb, out2, 1, cfl, status);
    return hipGetLastError();
}

// per-instance CFL wave speed of a batch of 2D instances (eq cfl for each):
// block (b, j0, j1) reduces rows j0..j1-1 of instance b; a second pass
// reduces each instance's blocks in a fixed order.
template <int N>
__global__ void k_wavespeed_batched(Phys ph, const Geo* __restrict__ geos, const int4* __restrict__ wl,
                                    const double* const* __restrict__ JUt,
                                    const double* const* __restrict__ Jt,
                                    const double* const* __restrict__ jxxt, double* __restrict__ part,
                                    unsigned* __restrict__ status)
{
    constexpr int D = 2;
    const int4 e = wl[blockIdx.x];
    const Geo g = geos[e.x];
    const double* JU = JUt[e.x];
    const double* Jv = Jt[e.x];
    const double* jxx = jxxt[e.x];
    const long P = g.P;
    const int n0 = g.n[0];
    const int cnt = (e.z - e.y) * n0;
    double lam = 0.0;
    unsigned bad = 0;
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
        const long i = node_index(g, q % n0 + g.ng, e.y + q / n0 + g.ng, 0);
        NodeState<N, D> s;
        load_state<N, D>(ph, JU, Jv, P, i, s);
        if (!s.ok) bad |= 1u;
        double cvr = 0.0, cg = 0.0, rR = 0.0;
#pragma unroll
        for (int l = 0; l < N; l++) {
            cvr += ph.cv[l] * s.U[l];
            cg += ph.cvgam[l] * s.U[l];
            rR += ph.Rg[l] * s.U[l];
        }
        const double c = sqrt((rR / s.rho) * (cg / cvr) * s.T);
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            double vn = 0.0, nn = 0.0;
#pragma unroll
            for (int j = 0; j < D; j++) {
                const double n = jxx[(k * D + j) * P + i];
                vn += s.v[j] * n;
                nn += n * n;
            }
            sum += (fabs(vn) + c * sqrt(nn)) / Jv[i] / g.dxi[k];
        }
        lam = fmax(lam, sum);
    }
    if (bad) atomicOr(status, bad);
    lam = block_reduce<RED_MAX>(lam);
    if (threadIdx.x == 0) part[blockIdx.x] = lam;
}

__global__ void k_finish_batched(const double* __restrict__ part, const int* __restrict__ first, double cfl,
                                 double* __restrict__ lam_out, double* __restrict__ dt_out)
{
    const int b = blockIdx.x;
    double v = -INFINITY;
    for (int t = first[b] + threadIdx.x; t < first[b + 1]; t += blockDim.x) v = fmax(v, part[t]);
    v = block_reduce<RED_MAX>(v);
    if (threadIdx.x == 0) {
        if (lam_out) lam_out[b] = v;
        dt_out[b] = cfl / v;
    }
}

hipError_t wavespeed_batched(const Phys& ph, const Geo* geos, const int4* wl, int nwl, const int* first,
                             int count, const double* const* JU, const double* const* J,
                             const double* const* jxx, double cfl, double* part, double* lambda_out,
                             double* dt_out, unsigned* status, hipStream_t s)
{
    if (ph.nspec == 1)
        hipLaunchKernelGGL(k_wavespeed_batched<1>, dim3(nwl), dim3(256), 0, s, ph, geos, wl, JU, J, jxx,
                           part, status);
    else
        hipLaunchKernelGGL(k_wavespeed_batched<2>, dim3(nwl), dim3(256), 0, s, ph, geos, wl, JU, J, jxx,
                           part, status);
    hipLaunchKernelGGL(k_finish_batched, dim3(count), dim3(256), 0, s, part, first, cfl, lambda_out, dt_out);
    return hipGetLastError();
}

template <int N, int D>
static void launch_entropy(const Phys& ph, const Geo& g, const double* JU, const double* J,
                           const double* dJU, const double* dJ, double* part, int nb, hipStream_t s)
{
    hipLaunchKernelGGL((k_entropy<N, D>), dim3(nb), dim3(256), 0, s, ph, g, JU, J, dJU, dJ, part);
}

hipError_t entropy_sum(const Phys& ph, const Geo& g, const double* JU, const double* J, const double* dJU,
                       const double* dJ, double* part, double* out, hipStream_t s)
{
    const long nint = (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
    const int nb = red_grid(nint);
    double dv = 1.0;
    for (int k = 0; k < g.dim; k++) dv *= g.dxi[k];
    ES_DISPATCH_ND(ph, g, launch_entropy, ph, g, JU, J, dJU, dJ, part, nb, s);
    hipLaunchKernelGGL(k_finish<RED_SUM>, dim3(1), dim3(256), 0, s, part, nb, out, 3, dv, nullptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// mesh redistribution (Section 4)
// ---------------------------------------------------------------------------
// |grad_xi sigma| by second-order central differences, for each monitor
// variable; per-block maxima into part[s * RED_BLOCKS + block].  The form
// with a Laplacian term also writes |lap_xi sigma| (second-order central
// differences) as channel nsig + s.  Variables: 0 rho, 1 rho_1, 2 rho_2,
// 3 p, 4 the speed |v| (the u of Example 5.9's monitor), 5 the schlieren
// function of eq schlieren, read from its array (with ghost layers).
// monitor variable sig at node i.  SIG: which variables the monitor may
// use, so that the kernels carry only the code (and registers) they need:
// 0 the densities (rho, rho_1, rho_2), 1 also the pressure, 2 also the
// speed and the schlieren function
template <int N, int D, int SIG = 0>
__device__ __forceinline__ double sigma_of(const Phys& ph, const double* JU, const double* Jv, long P,
                                           long i, int sig, const double* phi)
{
    if (SIG == 2 && sig == 5) return phi[i];
    const double Jq = Jv[i];
    if (SIG == 2 && sig == 4) {
        double r = 0.0, m2 = 0.0;
#pragma unroll
        for (int l = 0; l < N; l++) r += JU[l * P + i] / Jq;
#pragma unroll
        for (int j = 0; j < D; j++) {
            const double vj = (JU[(N + j) * P + i] / Jq) / r;
            m2 += vj * vj;
        }
        return sqrt(m2);
    }
    // (divisions, not a reciprocal of J: with the reciprocal the 3D gradient
    // took 310 instead of 240 us although it issues fewer instructions)
    if (sig == 0) {
        double r = 0.0;
#pragma unroll
        for (int l = 0; l < N; l++) r += JU[l * P + i] / Jq;
        return r;
    }
    if (sig == 1) return JU[i] / Jq;
    if (sig == 2 || SIG == 0) return JU[(N > 1 ? 1 : 0) * P + i] / Jq;
    NodeState<N, D> s;
    load_state<N, D>(ph, JU, Jv, P, i, s);
    return s.p;
}

template <int N, int D, int SIG>
__global__ void k_monitor_grad(Phys ph, Geo g, MonitorP mo, const double* __restrict__ JU,
                               const double* __restrict__ Jv, double* __restrict__ grad,
                               double* __restrict__ part)
{
    const long P = g.P;
    const long nint = n_interior(g);
    double gm[MON_CH] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        for (int s = 0; s < mo.nsig; s++) {
            double g2 = 0.0, lap = 0.0;
            const double sc = mo.form ? sigma_of<N, D, SIG>(ph, JU, Jv, P, i, mo.sigma[s], mo.phi) : 0.0;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const long st = dir_stride(g, k);
                const double sp = sigma_of<N, D, SIG>(ph, JU, Jv, P, i + st, mo.sigma[s], mo.phi);
                const double sm = sigma_of<N, D, SIG>(ph, JU, Jv, P, i - st, mo.sigma[s], mo.phi);
                const double dk = (sp - sm) / (2.0 * g.dxi[k]);
                g2 += dk * dk;
                lap += (sp - 2.0 * sc + sm) / (g.dxi[k] * g.dxi[k]);
            }
            const double gv = sqrt(g2);
            grad[s * P + i] = gv;
            gm[s] = fmax(gm[s], gv);
            if (mo.form) {
                grad[(mo.nsig + s) * P + i] = fabs(lap);
                gm[mo.nsig + s] = fmax(gm[mo.nsig + s], fabs(lap));
            }
        }
    }
    const int nch = mo.form ? 2 * mo.nsig : mo.nsig;
    for (int s = 0; s < MON_CH; s++) {
        if (s >= nch) break;   // uniform across the block
        const double r = block_reduce<RED_MAX>(gm[s]);
        if (threadIdx.x == 0) part[s * RED_BLOCKS + blockIdx.x] = r;
    }
}

// 3D monitor gradient walking z (the central differences of k_monitor_grad):
// each thread owns one (x, y) column of a 64 x 4 block over a chunk of z
// planes.  Sigma is evaluated once per node of each plane of the tile plus
// a 1-node in-plane halo (corners excepted) into a two-plane LDS buffer, so
// the in-plane neighbours and the plane above come from LDS and sigma at
// z-1 from a register: 1.5 evaluations per node instead of 5.
// Per-block maxima go to part[s * RED_BLOCKS + block] in block order.
template <int N, int SIG>
__global__ void __launch_bounds__(256)
k_monitor_grad3(Phys ph, Geo g, MonitorP mo, const double* __restrict__ JU, const double* __restrict__ Jv,
                double* __restrict__ grad, double* __restrict__ part, int zchunk)
{
    constexpr int D = 3;
    __shared__ double Sg[2][6][66];
    const long P = g.P;
    const int np0 = g.np[0], np1 = g.np[1];
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    const int lx = (int)(threadIdx.x & 63), ly = (int)(threadIdx.x >> 6);
    const int xt = g.ng + bx * 64, yt = g.ng + by * 4;
    const int x = xt + lx, y = yt + ly;
    const int zc0 = g.ng + bz * zchunk, zc1 = min(zc0 + zchunk, g.ng + g.n[2]);
    const bool in = x < g.ng + g.n[0] && y < g.ng + g.n[1];
    const long sz = (long)np0 * np1;
    double ih[3];
#pragma unroll
    for (int k = 0; k < 3; k++) ih[k] = 1.0 / (2.0 * g.dxi[k]);
    // sigma of channel sg at plane zz of the patch into buffer b
    auto stage = [&](int b, int zz, int sg) {
        for (int q = threadIdx.x; q < 6 * 66; q += 256) {
            const int hx = q % 66, hy = q / 66;
            const bool corner = (hx == 0 || hx == 65) && (hy == 0 || hy == 5);
            const int gx = xt - 1 + hx, gy = yt - 1 + hy;
            if (!corner && gx < np0 && gy < np1)
                Sg[b][hy][hx] = sigma_of<N, D, SIG>(ph, JU, Jv, P, ((long)zz * np1 + gy) * np0 + gx, sg, mo.phi);
        }
    };
    double gm[MON_CH] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (zc0 < zc1) {   // uniform over the block
        for (int s = 0; s < mo.nsig; s++) {
            const int sg = mo.sigma[s];
            long i = ((long)zc0 * np1 + y) * np0 + x;
            double sm = in ? sigma_of<N, D, SIG>(ph, JU, Jv, P, i - sz, sg, mo.phi) : 0.0;
            double mg = 0.0, ml = 0.0;     // this channel's maxima over the column
            int cur = 0;
            stage(cur, zc0, sg);
            for (int z = zc0; z < zc1; z++, i += sz) {
                stage(cur ^ 1, z + 1, sg);
                __syncthreads();
                if (in) {
                    const int hx = lx + 1, hy = ly + 1;
                    const double s0 = Sg[cur][hy][hx];
                    const double sp = Sg[cur ^ 1][hy][hx];
                    const double xp = Sg[cur][hy][hx + 1];
                    const double xm = Sg[cur][hy][hx - 1];
                    const double yp = Sg[cur][hy + 1][hx];
                    const double ym = Sg[cur][hy - 1][hx];
                    const double d0 = (xp - xm) * ih[0];
                    const double d1 = (yp - ym) * ih[1];
                    const double d2 = (sp - sm) * ih[2];
                    const double gv = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    grad[s * P + i] = gv;
                    mg = fmax(mg, gv);
                    if (mo.form) {   // the same sum as k_monitor_grad: directions 0, 1, 2 in order
                        double lap = (xp - 2.0 * s0 + xm) / (g.dxi[0] * g.dxi[0]);
                        lap += (yp - 2.0 * s0 + ym) / (g.dxi[1] * g.dxi[1]);
                        lap += (sp - 2.0 * s0 + sm) / (g.dxi[2] * g.dxi[2]);
                        grad[(mo.nsig + s) * P + i] = fabs(lap);
                        ml = fmax(ml, fabs(lap));
                    }
                    sm = s0;
                }
                __syncthreads();   // the next plane overwrites buffer cur
                cur ^= 1;
            }
#pragma unroll
            for (int c = 0; c < MON_CH; c++) {
                if (c == s) gm[c] = mg;
                if (mo.form && c == mo.nsig + s) gm[c] = ml;
            }
        }
    }
    const long blk = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int nch = mo.form ? 2 * mo.nsig : mo.nsig;
#pragma unroll
    for (int s = 0; s < MON_CH; s++) {
        const double r = block_reduce<RED_MAX>(gm[s]);
        if (threadIdx.x == 0 && s < nch) part[s * RED_BLOCKS + blk] = r;
    }
}

// 3D monitor filter walking z: the weights 2^-(|j|_1 + 3), j in {-1,0,1}^3,
// are the product of (1/4, 1/2, 1/4) along each direction, so each plane
// contributes its 9-point in-plane sum q(z') and out = q(z-1)/4 + q(z)/2 +
// q(z+1)/4 from a 3-plane ring.  The in-plane sums read the plane of the
// tile plus a 1-node halo staged in LDS.
__global__ void __launch_bounds__(256)
k_filter3(Geo g, const double* __restrict__ in, double* __restrict__ out, int zchunk)
{
    __shared__ double Fs[6][66];
    const int np0 = g.np[0], np1 = g.np[1];
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    const int lx = (int)(threadIdx.x & 63), ly = (int)(threadIdx.x >> 6);
    const int xt = g.ng + bx * 64, yt = g.ng + by * 4;
    const int x = xt + lx, y = yt + ly;
    const int zc0 = g.ng + bz * zchunk, zc1 = min(zc0 + zchunk, g.ng + g.n[2]);
    if (zc0 >= zc1) return;   // uniform over the block
    const bool inside = x < g.ng + g.n[0] && y < g.ng + g.n[1];
    const long sz = (long)np0 * np1;
    auto stage = [&](int zz) {
        for (int q = threadIdx.x; q < 6 * 66; q += 256) {
            const int hx = q % 66, hy = q / 66;
            const int gx = xt - 1 + hx, gy = yt - 1 + hy;
            if (gx < np0 && gy < np1) Fs[hy][hx] = in[((long)zz * np1 + gy) * np0 + gx];
        }
    };
    auto plane = [&]() {   // in-plane (1/4, 1/2, 1/4) x (1/4, 1/2, 1/4) sum around the own node
        const int hx = lx + 1, hy = ly + 1;
        const double r0 = 0.25 * Fs[hy - 1][hx - 1] + 0.5 * Fs[hy - 1][hx] + 0.25 * Fs[hy - 1][hx + 1];
        const double r1 = 0.25 * Fs[hy][hx - 1] + 0.5 * Fs[hy][hx] + 0.25 * Fs[hy][hx + 1];
        const double r2 = 0.25 * Fs[hy + 1][hx - 1] + 0.5 * Fs[hy + 1][hx] + 0.25 * Fs[hy + 1][hx + 1];
        return 0.25 * r0 + 0.5 * r1 + 0.25 * r2;
    };
    long i = ((long)zc0 * np1 + y) * np0 + x;
    double qm = 0.0, q0 = 0.0;
    stage(zc0 - 1);
    __syncthreads();
    if (inside) qm = plane();
    __syncthreads();
    stage(zc0);
    __syncthreads();
    if (inside) q0 = plane();
    __syncthreads();
    for (int z = zc0; z < zc1; z++, i += sz) {
        stage(z + 1);
        __syncthreads();
        if (inside) {
            const double qp = plane();
            out[i] = 0.25 * qm + 0.5 * q0 + 0.25 * qp;
            qm = q0;
            q0 = qp;
        }
        __syncthreads();
    }
}

// the schlieren function of eq schlieren, Phi = exp(-Psi |grad rho| /
// max |grad rho|), Psi = (psi_1 rho_1 + psi_2 rho_2) / rho: first
// |grad_xi rho| (the monitor's central differences) with per-block maxima,
// then Phi from the global maximum (1 where it is 0)
template <int N, int D>
__global__ void k_rho_grad(Phys ph, Geo g, const double* __restrict__ JU, const double* __restrict__ Jv,
                           double* __restrict__ gr, double* __restrict__ part)
{
    const long P = g.P;
    const long nint = n_interior(g);
    double gm = 0.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        double g2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            const long st = dir_stride(g, k);
            const double sp = sigma_of<N, D>(ph, JU, Jv, P, i + st, 0, nullptr);
            const double sm = sigma_of<N, D>(ph, JU, Jv, P, i - st, 0, nullptr);
            const double dk = (sp - sm) / (2.0 * g.dxi[k]);
            g2 += dk * dk;
        }
        gr[i] = sqrt(g2);
        gm = fmax(gm, gr[i]);
    }
    const double r = block_reduce<RED_MAX>(gm);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

template <int N, int D>
__global__ void k_schlieren(Phys ph, Geo g, MonitorP mo, const double* __restrict__ JU,
                            const double* __restrict__ Jv, const double* __restrict__ gr,
                            const double* __restrict__ gmax, double* __restrict__ phi)
{
    const long P = g.P;
    const long nint = n_interior(g);
    const double G = *gmax;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        double psi = mo.psi[0];
        if (N == 2) {
            const double r1 = sigma_of<N, D>(ph, JU, Jv, P, i, 1, nullptr);
            const double r = sigma_of<N, D>(ph, JU, Jv, P, i, 0, nullptr);
            psi = (mo.psi[0] * r1 + mo.psi[1] * (r - r1)) / r;
        }
        phi[i] = G > 0.0 ? exp(-psi * gr[i] / G) : 1.0;
    }
}

template <int N, int D>
static void launch_schlieren(const Phys& ph, const Geo& g, const MonitorP& mo, const double* JU,
                             const double* J, double* gr, double* part, double* gmax, double* phi, int nb,
                             int gi, hipStream_t s)
{
    hipLaunchKernelGGL((k_rho_grad<N, D>), dim3(nb), dim3(256), 0, s, ph, g, JU, J, gr, part);
    hipLaunchKernelGGL(k_finish<RED_MAX>, dim3(1), dim3(256), 0, s, part, nb, gmax, 0, 0.0, nullptr);
    hipLaunchKernelGGL((k_schlieren<N, D>), dim3(gi), dim3(256), 0, s, ph, g, mo, JU, J, gr, gmax, phi);
}

__device__ __forceinline__ double theta_node(const MonitorP& mo, const double* grad, const double* gmax, long P,
                                             long i)
{
    double th = 1.0;
    for (int s = 0; s < mo.nsig; s++) {
        const double G = gmax[s];
        if (G > 0.0) {
            const double r = grad[s * P + i] / G;
            th += mo.form ? mo.alpha[s] * r : mo.alpha[s] * r * r;
        }
        if (mo.form && gmax[mo.nsig + s] > 0.0)
            th += mo.beta[s] * (grad[(mo.nsig + s) * P + i] / gmax[mo.nsig + s]);
    }
    return sqrt(th);
}

__global__ void k_theta(Geo g, MonitorP mo, const double* __restrict__ grad, const double* __restrict__ gmax,
                        double* __restrict__ theta, long nzs, long nys, long nxs)
{
    const long P = g.P;
    const long nint = n_interior(g);
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        theta[i] = theta_node(mo, grad, gmax, P, i);
    }
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nzs + nys + nxs;
         t += (long)gridDim.x * blockDim.x) {
        int side[3];
        long di;
        const long si = shell_image(g, t, nzs, nys, side, di);
        theta[di] = theta_node(mo, grad, gmax, P, si);
    }
}

// low-pass filter: sum over j in {0,+-1}^d of (1/2)^(|j|_1 + d) Theta_{i+j}
__device__ __forceinline__ double filter_node(const Geo& g, const double* in, long i)
{
    const long s0 = 1, s1 = g.np[0], s2 = (long)g.np[0] * g.np[1];
    const int r2 = g.dim == 3 ? 1 : 0;
    double s = 0.0;
    for (int j2 = -r2; j2 <= r2; j2++)
        for (int j1 = -1; j1 <= 1; j1++)
            for (int j0 = -1; j0 <= 1; j0++) {
                const int e = abs(j0) + abs(j1) + abs(j2) + g.dim;
                s += ldexp(1.0, -e) * in[i + j0 * s0 + j1 * s1 + j2 * s2];
            }
    return s;
}

__global__ void k_filter(Geo g, const double* __restrict__ in, double* __restrict__ out, long nzs, long nys,
                         long nxs)
{
    const long nint = n_interior(g);
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        out[i] = filter_node(g, in, i);
    }
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nzs + nys + nxs;
         t += (long)gridDim.x * blockDim.x) {
        int side[3];
        long di;
        const long si = shell_image(g, t, nzs, nys, side, di);
        out[di] = filter_node(g, in, si);
    }
}

// one Jacobi update of interior node i
template <int D>
__device__ __forceinline__ void jacobi_node(const Geo& g, const double* th, const double* xa, long i, double* xn)
{
    // Theta_{k+-1/2} / dxi_k^2, and one reciprocal of the denominator the D
    // coordinates share
    const long P = g.P;
    double tp[D], tm[D];
    double den = 0.0;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const long st = dir_stride(g, k);
        const double w2 = 1.0 / (g.dxi[k] * g.dxi[k]);
        tp[k] = 0.5 * (th[i] + th[i + st]);
        tm[k] = 0.5 * (th[i] + th[i - st]);
        tp[k] *= w2;
        tm[k] *= w2;
        den += tp[k] + tm[k];
    }
    const double iden = rcp(den);
#pragma unroll
    for (int c = 0; c < D; c++) {
        double num = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            const long st = dir_stride(g, k);
            num += tp[k] * xa[c * P + i + st] + tm[k] * xa[c * P + i - st];
        }
        xn[c] = num * iden;
    }
}

// one Jacobi sweep of the mesh equations, per-block max |x_new - x_old|,
// with the ghost layers of its output in the same launch: a
// ghost node takes the update of the interior node it wraps or mirrors to
// (computed again, with the same arithmetic) under the mesh's ghost rule
template <int D>
__global__ void k_jacobi(Geo g, const double* __restrict__ th, const double* __restrict__ xa,
                         double* __restrict__ xb, double* __restrict__ part, long nzs, long nys, long nxs)
{
    const long P = g.P;
    const long nint = n_interior(g);
    double r = 0.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        double xn[D];
        jacobi_node<D>(g, th, xa, i, xn);
#pragma unroll
        for (int c = 0; c < D; c++) {
            xb[c * P + i] = xn[c];
            r = fmax(r, fabs(xn[c] - xa[c * P + i]));
        }
    }
    const long total = nzs + nys + nxs;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        int d[3];
        shell_node(g, t, nzs, nys, d);
        int sidx[3] = {d[0], d[1], d[2]}, side[3] = {0, 0, 0};
        for (int k = 0; k < D; k++) sidx[k] = ghost_image(g, k, d[k], side[k]);
        double xn[D];
        jacobi_node<D>(g, th, xa, node_index(g, sidx[0], sidx[1], sidx[2]), xn);
        const long di = node_index(g, d[0], d[1], d[2]);
#pragma unroll
        for (int c = 0; c < D; c++) xb[c * P + di] = ghost_value(g, GH_MESH, c, side, xn[c]);
    }
    r = block_reduce<RED_MAX>(r);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// 3D Jacobi sweep (the arithmetic of k_jacobi<3>, term for term), walking
// z: each thread owns one (x, y) column of a 64 x 4 block over a chunk of z
// planes; theta and x at z-1 and z+1 come from a 3-plane ring in registers,
// the in-plane neighbours from the plane's theta and x staged in LDS with a
// 1-node halo (reading them from the caches instead took 323 against 259 us
// at 256^3, with 106 registers and four waves per SIMD instead of eight).
// Per-block residual maxima go to part[] in block order.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_jacobi3(Geo g, const double* __restrict__ th, const double* __restrict__ xa, double* __restrict__ xb,
          double* __restrict__ part, int zchunk)
{
    // the plane's theta and x of the tile plus a 1-node in-plane halo
    __shared__ double Ts[6][66];
    __shared__ double Xs[3][6][66];
    const long P = g.P;
    const int np0 = g.np[0], np1 = g.np[1];
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    const int lx = (int)(threadIdx.x & 63), ly = (int)(threadIdx.x >> 6);
    const int xt = g.ng + bx * 64, yt = g.ng + by * 4;
    const int x = xt + lx, y = yt + ly;
    const int zc0 = g.ng + bz * zchunk, zc1 = min(zc0 + zchunk, g.ng + g.n[2]);
    const bool in = x < g.ng + g.n[0] && y < g.ng + g.n[1];
    const long sz = (long)np0 * np1;
    double w2[3];
#pragma unroll
    for (int k = 0; k < 3; k++) w2[k] = 1.0 / (g.dxi[k] * g.dxi[k]);
    double r = 0.0;
    long i = ((long)zc0 * np1 + y) * np0 + x;
    double tm1 = 0.0, t0 = 0.0, xm1[3] = {0.0, 0.0, 0.0}, x0[3] = {0.0, 0.0, 0.0};
    if (in && zc0 < zc1) {
        tm1 = th[i - sz];
        t0 = th[i];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            xm1[c] = xa[c * P + i - sz];
            x0[c] = xa[c * P + i];
        }
    }
    for (int z = zc0; z < zc1; z++, i += sz) {
        for (int q = threadIdx.x; q < 6 * 66; q += 256) {
            const int hx = q % 66, hy = q / 66;
            const int gx = xt - 1 + hx, gy = yt - 1 + hy;
            if (gx < np0 && gy < np1) {
                const long gi = ((long)z * np1 + gy) * np0 + gx;
                Ts[hy][hx] = th[gi];
#pragma unroll
                for (int c = 0; c < 3; c++) Xs[c][hy][hx] = xa[c * P + gi];
            }
        }
        __syncthreads();
        if (in) {
            const double tp1 = th[i + sz];
            double xp1[3];
#pragma unroll
            for (int c = 0; c < 3; c++) xp1[c] = xa[c * P + i + sz];
            const int hx = lx + 1, hy = ly + 1;
            double tp[3], tm[3];
            tp[0] = 0.5 * (t0 + Ts[hy][hx + 1]);
            tm[0] = 0.5 * (t0 + Ts[hy][hx - 1]);
            tp[1] = 0.5 * (t0 + Ts[hy + 1][hx]);
            tm[1] = 0.5 * (t0 + Ts[hy - 1][hx]);
            tp[2] = 0.5 * (t0 + tp1);
            tm[2] = 0.5 * (t0 + tm1);
            double den = 0.0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                tp[k] *= w2[k];
                tm[k] *= w2[k];
                den += tp[k] + tm[k];
            }
            const double iden = rcp(den);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                double num = tp[0] * Xs[c][hy][hx + 1] + tm[0] * Xs[c][hy][hx - 1];
                num += tp[1] * Xs[c][hy + 1][hx] + tm[1] * Xs[c][hy - 1][hx];
                num += tp[2] * xp1[c] + tm[2] * xm1[c];
                const double xn = num * iden;
                xb[c * P + i] = xn;
                r = fmax(r, fabs(xn - x0[c]));
            }
            tm1 = t0;
            t0 = tp1;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                xm1[c] = x0[c];
                x0[c] = xp1[c];
            }
        }
        __syncthreads();
    }
    r = block_reduce<RED_MAX>(r);
    if (threadIdx.x == 0) part[((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = r;
}

// movement limiter: per-block min of the bounds (1 if none)
template <int D>
__global__ void k_limiter(Geo g, const double* __restrict__ xmu, const double* __restrict__ xn,
                          double* __restrict__ part)
{
    const long P = g.P;
    const long nint = n_interior(g);
    double b = 1.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
#pragma unroll
        for (int k = 0; k < D; k++) {
            const long st = dir_stride(g, k);
            const double dx = xmu[k * P + i] - xn[k * P + i];
            if (dx < 0.0) b = fmin(b, -(xn[k * P + i] - xn[k * P + i - st]) / (2.0 * dx));
            else if (dx > 0.0) b = fmin(b, (xn[k * P + i + st] - xn[k * P + i]) / (2.0 * dx));
        }
    }
    b = block_reduce<RED_MIN>(b);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// disp = Delta_tau (x^[mu] - x_n) with its ghost layers; with xnext, also
// x_{n+1} = x_n + disp with the mesh's ghost layers (each ghost node from
// the sum at its image node, as a ghost fill of x_{n+1} gives it)
__global__ void k_disp(Geo g, const double* __restrict__ xmu, const double* __restrict__ xn,
                       const double* __restrict__ dtau, double* __restrict__ disp, double* __restrict__ xnext,
                       long nzs, long nys, long nxs)
{
    const long P = g.P;
    const long nint = n_interior(g);
    const double d = *dtau;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nint; q += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        const long i = interior_node(g, q, i0, i1, i2);
        for (int c = 0; c < g.dim; c++) {
            const double v = d * (xmu[c * P + i] - xn[c * P + i]);
            disp[c * P + i] = v;
            if (xnext) xnext[c * P + i] = xn[c * P + i] + v;
        }
    }
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nzs + nys + nxs;
         t += (long)gridDim.x * blockDim.x) {
        int side[3];
        long di;
        const long si = shell_image(g, t, nzs, nys, side, di);
        for (int c = 0; c < g.dim; c++) {
            const double v = d * (xmu[c * P + si] - xn[c * P + si]);
            disp[c * P + di] = ghost_value(g, GH_DISP, c, side, v);
            if (xnext) xnext[c * P + di] = ghost_value(g, GH_MESH, c, side, xn[c * P + si] + v);
        }
    }
}

template <int N, int D>
static void launch_monitor(const Phys& ph, const Geo& g, const MonitorP& mo, int sigmode, const double* JU,
                           const double* J, double* grad, double* part, int nb, hipStream_t s)
{
    if (sigmode == 2)
        hipLaunchKernelGGL((k_monitor_grad<N, D, 2>), dim3(nb), dim3(256), 0, s, ph, g, mo, JU, J, grad, part);
    else if (sigmode == 1)
        hipLaunchKernelGGL((k_monitor_grad<N, D, 1>), dim3(nb), dim3(256), 0, s, ph, g, mo, JU, J, grad, part);
    else
        hipLaunchKernelGGL((k_monitor_grad<N, D, 0>), dim3(nb), dim3(256), 0, s, ph, g, mo, JU, J, grad, part);
}

hipError_t mesh_redistribute(const Phys& ph, const Geo& g, const MonitorP& mo_in, const double* JU,
                             const double* J, const double* xn, double* disp, MeshWork& w,
                             double* dtau_out, double* resid_out, unsigned* status, hipStream_t s,
                             double* xnext)
{
    MonitorP mo = mo_in;
    mo.phi = w.phi;
    const long P = g.P;
    const long nint = (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
    const int nb = red_grid(nint);
    const int gi = grid_for(nint);
    // 3D kernels walk z over 64 x 4 columns, in z chunks so that the blocks
    // (one reduction partial each) stay within the partial buffer
    const int jx = (g.n[0] + 63) / 64, jy = (g.n[1] + 3) / 4;
    const int jz = std::max(1, std::min(g.n[2], RED_BLOCKS / (jx * jy)));
    const int jchunk = (g.n[2] + jz - 1) / jz;
    const dim3 jgrid(jx, jy, (g.n[2] + jchunk - 1) / jchunk);
    const int jblocks = jx * jy * (int)jgrid.z;
    const bool march = g.dim == 3 && jblocks <= RED_BLOCKS;
    // the schlieren function first when the monitor uses it (th1 holds
    // |grad rho| until the filter overwrites it)
    bool use_phi = false, ext = false, press = false;
    for (int q = 0; q < mo.nsig; q++) {
        use_phi = use_phi || mo.sigma[q] == 5;
        ext = ext || mo.sigma[q] >= 4;
        press = press || mo.sigma[q] == 3;
    }
    // the monitor kernels carry only the variables they are asked for
    const int sigmode = ext ? 2 : (press ? 1 : 0);
    if (use_phi) {
        ES_DISPATCH_ND(ph, g, launch_schlieren, ph, g, mo, JU, J, w.th1, w.part + 6 * RED_BLOCKS, w.scal + 7,
                       w.phi, nb, gi, s);
        const hipError_t e0 = fill_ghosts(g, w.phi, 1, GH_PLAIN, s);
        if (e0 != hipSuccess) return e0;
    }
    // monitor and its global maxima
    if (march) {
        auto* kern = ph.nspec == 1
                         ? (sigmode == 2 ? k_monitor_grad3<1, 2> : (sigmode == 1 ? k_monitor_grad3<1, 1> : k_monitor_grad3<1, 0>))
                         : (sigmode == 2 ? k_monitor_grad3<2, 2> : (sigmode == 1 ? k_monitor_grad3<2, 1> : k_monitor_grad3<2, 0>));
        hipLaunchKernelGGL(kern, jgrid, dim3(256), 0, s, ph, g, mo, JU, J, w.grad, w.part, jchunk);
    } else {
        ES_DISPATCH_ND(ph, g, launch_monitor, ph, g, mo, sigmode, JU, J, w.grad, w.part, nb, s);
    }
    for (int q = 0; q < (mo.form ? 2 * mo.nsig : mo.nsig); q++)
        hipLaunchKernelGGL(k_finish<RED_MAX>, dim3(1), dim3(256), 0, s, w.part + q * RED_BLOCKS,
                           march ? jblocks : nb, w.scal + q, 0, 0.0, status);
    // theta, the filter passes that are not z-marching, the Jacobi sweeps
    // that are not and the displacement write their own ghost layers
    long nzs, nys, nxs;
    shell_sizes(g, nzs, nys, nxs);
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_theta, dim3(gi), dim3(256), 0, s, g, mo, w.grad, w.scal, w.th0, nzs, nys, nxs);
    double* th = w.th0;
    double* th2 = w.th1;
    for (int q = 0; q < mo.n_smooth; q++) {
        if (march) {
            hipLaunchKernelGGL(k_filter3, jgrid, dim3(256), 0, s, g, th, th2, jchunk);
            if ((e = fill_ghosts(g, th2, 1, GH_PLAIN, s)) != hipSuccess) return e;
        } else {
            hipLaunchKernelGGL(k_filter, dim3(gi), dim3(256), 0, s, g, th, th2, nzs, nys, nxs);
        }
        std::swap(th, th2);
    }
    // Jacobi sweeps: the first reads x_n itself, then xa and xb alternate
    const double* xcur = xn;
    double* xa = w.xa;
    double* xb = w.xb;
    for (int nu = 0; nu < mo.n_sweeps; nu++) {
        if (march)
            hipLaunchKernelGGL(k_jacobi3, jgrid, dim3(256), 0, s, g, th, xcur, xa, w.part, jchunk);
        else if (g.dim == 2)
            hipLaunchKernelGGL(k_jacobi<2>, dim3(nb), dim3(256), 0, s, g, th, xcur, xa, w.part, nzs, nys, nxs);
        else
            hipLaunchKernelGGL(k_jacobi<3>, dim3(nb), dim3(256), 0, s, g, th, xcur, xa, w.part, nzs, nys, nxs);
        if (march && (e = fill_ghosts(g, xa, g.dim, GH_MESH, s)) != hipSuccess) return e;
        if (resid_out)
            hipLaunchKernelGGL(k_finish<RED_MAX>, dim3(1), dim3(256), 0, s, w.part, march ? jblocks : nb,
                               resid_out + nu, 0, 0.0, status);
        xcur = xa;
        std::swap(xa, xb);
    }
    // limiter and displacement
    if (g.dim == 2)
        hipLaunchKernelGGL(k_limiter<2>, dim3(nb), dim3(256), 0, s, g, xcur, xn, w.part);
    else
        hipLaunchKernelGGL(k_limiter<3>, dim3(nb), dim3(256), 0, s, g, xcur, xn, w.part);
    hipLaunchKernelGGL(k_finish<RED_MIN>, dim3(1), dim3(256), 0, s, w.part, nb, w.scal + 6, 2, 0.0, status);
    hipLaunchKernelGGL(k_disp, dim3(gi), dim3(256), 0, s, g, xcur, xn, w.scal + 6, disp, xnext, nzs, nys, nxs);
    if (dtau_out && (e = copy(w.scal + 6, dtau_out, 1, s)) != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace es
