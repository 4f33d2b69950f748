// LPT kernels for gfx950 (Hahn & Abel 2011, Section 3.1, and the baryon density of Section 5.3):
//   first order   psi_c = scale * G_c phi            (Table 1 gradient, fourth or sixth order)
//   second order  tau = sum_{i>j} D_ii D_jj - D_ij^2,  D_ij = G_i (G_j phi)
//   LLA density   rho / rho_bar - 1 = 1 / det(I + G4 L) - 1   (eq. gasdens)
// plus the post-solve ghost layers of width R (faces, edges and corners) that patches need:
// coarse-only tri-quadratic interpolation of the parent at the child's position (children sit at
// -1/4 and +1/4 of the parent cell along each axis).
//
// Sources are either periodic n^3 arrays (indices wrap) or arrays padded by R ghost cells on
// every side; the two cases are separate instantiations.  The gradient is evaluated as
// ((u[-2] - 8 u[-1]) + 8 u[+1]) - u[+2], / (12 h), then scaled.  tau takes two passes:
// psi_j = G4_j phi is stored (extended by 2 cells on patches), then D_ij = G4_i psi_j is
// evaluated per cell.  Output cells are decoded from a linear index with multiply-shift
// division (every array has fewer than 2^31 cells).  Periodic levels take groups of rows, and
// where the tile divides the level, x-marched tiles with a ring of plane slabs in LDS.

#include "mg_internal.h"

namespace mgic {

template <bool PAD>
struct Src {
    const double* p;
    int R;    // padding (PAD) - unused when periodic
    Dims d;   // interior dims
    __device__ __forceinline__ double at(int x, int y, int z) const {
        if constexpr (!PAD) {
            x = x < 0 ? x + d.x : (x >= d.x ? x - d.x : x);
            y = y < 0 ? y + d.y : (y >= d.y ? y - d.y : y);
            z = z < 0 ? z + d.z : (z >= d.z ? z - d.z : z);
            return p[((unsigned)x * d.y + y) * (unsigned)d.z + z];
        } else {
            const unsigned py = (unsigned)d.y + 2 * R, pz = (unsigned)d.z + 2 * R;
            return p[((unsigned)(x + R) * py + (y + R)) * pz + (z + R)];
        }
    }
};

// fourth-order gradient of s along `axis` at (x, y, z), Table 1 weights (1, -8, 0, 8, -1) / 12
template <bool PAD>
__device__ __forceinline__ double g4(const Src<PAD>& s, int x, int y, int z, int axis, double den) {
    const int ex = axis == 0, ey = axis == 1, ez = axis == 2;
    double acc = s.at(x - 2 * ex, y - 2 * ey, z - 2 * ez);
    acc = acc + (-8.0) * s.at(x - ex, y - ey, z - ez);
    acc = acc + 8.0 * s.at(x + ex, y + ey, z + ez);
    acc = acc + (-1.0) * s.at(x + 2 * ex, y + 2 * ey, z + 2 * ez);
    return acc / den;
}

// sixth-order gradient of s along `axis`, Table 1 weights (-1, 9, -45, 0, 45, -9, 1) / 60
template <bool PAD>
__device__ __forceinline__ double g6(const Src<PAD>& s, int x, int y, int z, int axis, double den) {
    const int ex = axis == 0, ey = axis == 1, ez = axis == 2;
    double acc = (-1.0) * s.at(x - 3 * ex, y - 3 * ey, z - 3 * ez);
    acc = acc + 9.0 * s.at(x - 2 * ex, y - 2 * ey, z - 2 * ez);
    acc = acc + (-45.0) * s.at(x - ex, y - ey, z - ez);
    acc = acc + 45.0 * s.at(x + ex, y + ey, z + ez);
    acc = acc + (-9.0) * s.at(x + 2 * ex, y + 2 * ey, z + 2 * ez);
    acc = acc + s.at(x + 3 * ex, y + 3 * ey, z + 3 * ez);
    return acc / den;
}

// the gradient of order G (4 or 6) with its denominator (12 h or 60 h)
template <bool PAD, int G>
__device__ __forceinline__ double gG(const Src<PAD>& s, int x, int y, int z, int axis, double h) {
    if constexpr (G == 4) return g4(s, x, y, z, axis, 12.0 * h);
    else return g6(s, x, y, z, axis, 60.0 * h);
}

// linear index -> (x, y, z) of a box, natural order
__device__ __forceinline__ void decode3(const Lay& B, unsigned t, int& x, int& y, int& z) {
    const unsigned row = B.dz.div(t);
    z = (int)(t - row * (unsigned)B.d.z);
    const unsigned xq = B.dy.div(row);
    y = (int)(row - xq * (unsigned)B.d.y);
    x = (int)xq;
}

template <bool PAD, int G = 4>
__global__ void k_grad4(Src<PAD> s, Lay B, double h, double scale, double* __restrict__ ox,
                        double* __restrict__ oy, double* __restrict__ oz) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int x, y, z;
    decode3(B, t, x, y, z);
    ox[t] = scale * gG<PAD, G>(s, x, y, z, 0, h);
    oy[t] = scale * gG<PAD, G>(s, x, y, z, 1, h);
    oz[t] = scale * gG<PAD, G>(s, x, y, z, 2, h);
}

// psi_j = G_j phi on the interior extended by e cells (e <= R - G / 2), unscaled; the output box
// B is (d + 2e)^3, padded by e
template <bool PAD, int G = 4>
__global__ void k_psi(Src<PAD> s, Lay B, int e, double h, double* __restrict__ p0, double* __restrict__ p1,
                      double* __restrict__ p2) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int x, y, z;
    decode3(B, t, x, y, z);
    x -= e;
    y -= e;
    z -= e;
    p0[t] = gG<PAD, G>(s, x, y, z, 0, h);
    p1[t] = gG<PAD, G>(s, x, y, z, 1, h);
    p2[t] = gG<PAD, G>(s, x, y, z, 2, h);
}

// tau = sum_{i>j} D_ii D_jj - D_ij^2 with D_ij = G_i psi_j; psi periodic or padded by e.  When
// psi is a scaled gradient s G phi, post = 1 / s^2 brings tau back to the one of phi (post = 1:
// not applied, so s = +-1 gives the same bits as psi = G phi)
template <bool PAD, int G = 4>
__global__ void k_tau_psi(Src<PAD> q0, Src<PAD> q1, Src<PAD> q2, Lay B, double h, double post,
                          double* __restrict__ tau) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int x, y, z;
    decode3(B, t, x, y, z);
    const double Dxx = gG<PAD, G>(q0, x, y, z, 0, h);
    const double Dyy = gG<PAD, G>(q1, x, y, z, 1, h);
    const double Dzz = gG<PAD, G>(q2, x, y, z, 2, h);
    const double Dyx = gG<PAD, G>(q0, x, y, z, 1, h);
    const double Dzx = gG<PAD, G>(q0, x, y, z, 2, h);
    const double Dzy = gG<PAD, G>(q1, x, y, z, 2, h);
    double acc = 0.0;
    acc = acc + (Dyy * Dxx - Dyx * Dyx);
    acc = acc + (Dzz * Dxx - Dzx * Dzx);
    acc = acc + (Dzz * Dyy - Dzy * Dzy);
    tau[t] = post == 1.0 ? acc : acc * post;
}

// LLA baryon density (Section 5.3, eq. gasdens): rho / rho_bar - 1 = 1 / det(I + J) - 1 with
// J_ij = G4_j L_i, where the displacement L is a (+ b when `sum`, formed per load, the same
// add a separate pass would make).  The stencil sums are multiplied by 1 / (12 h) (as g4m), and
// the determinant is expanded along the first row of M = I + J.
template <bool PAD>
__device__ __forceinline__ double g4_of(const Src<PAD>& a, const Src<PAD>& b, int sum, int x, int y, int z,
                                        int axis, double inv) {
    const int ex = axis == 0, ey = axis == 1, ez = axis == 2;
    auto v = [&](int k) {
        const int X = x + k * ex, Y = y + k * ey, Z = z + k * ez;
        return sum ? a.at(X, Y, Z) + b.at(X, Y, Z) : a.at(X, Y, Z);
    };
    double acc = v(-2);
    acc = acc + (-8.0) * v(-1);
    acc = acc + 8.0 * v(1);
    acc = acc + (-1.0) * v(2);
    return acc * inv;
}

template <bool PAD>
__global__ void k_lla(Src<PAD> a0, Src<PAD> a1, Src<PAD> a2, Src<PAD> b0, Src<PAD> b1, Src<PAD> b2, int sum,
                      Lay B, double h, double* __restrict__ out) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int x, y, z;
    decode3(B, t, x, y, z);
    const double inv = 1.0 / (12.0 * h);
    const Src<PAD>* A[3] = {&a0, &a1, &a2};
    const Src<PAD>* Bs[3] = {&b0, &b1, &b2};
    double m[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m[i][j] = (i == j ? 1.0 : 0.0) + g4_of(*A[i], *Bs[i], sum, x, y, z, j, inv);
    const double c0 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    const double c1 = m[1][0] * m[2][2] - m[1][2] * m[2][0];
    const double c2 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    const double det = (m[0][0] * c0 - m[0][1] * c1) + m[0][2] * c2;
    out[t] = 1.0 / det - 1.0;
}

__global__ void k_add2(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ dst, size_t n) {
    for (size_t i = (size_t)lpt_block() * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = a[i] + b[i];
}

// ----------------------------------------------------------------------------------------------
// Periodic natural-order arrays, by groups of rows: one workgroup per (x, 8 consecutive y), each
// thread one z walking the 8 rows with the y-stencil values in a register window.  The blocks of
// one x plane are spread over the XCDs in turn, so with one block per row every row would be
// fetched into the L2 of each XCD whose rows are its y-neighbours; by groups, only the 4 halo rows
// of a group are shared with the two neighbouring groups, and the blocks of x-neighbouring planes
// (ng blocks apart) land on the same XCD whenever ng is a multiple of 8.  Same arithmetic as
// g4 (bit-identical results).
// ----------------------------------------------------------------------------------------------
constexpr int kRowsY = 8;

__device__ __forceinline__ double g4v(double m2, double m1, double p1, double p2, double den) {
    double acc = m2;
    acc = acc + (-8.0) * m1;
    acc = acc + 8.0 * p1;
    acc = acc + (-1.0) * p2;
    return acc / den;
}

// the G4 stencil of the LLA kernels: the same sum as g4v, times inv = 1 / (12 h) (a
// multiplication instead of nine divisions per cell)
__device__ __forceinline__ double g4m(double m2, double m1, double p1, double p2, double inv) {
    double acc = m2;
    acc = acc + (-8.0) * m1;
    acc = acc + 8.0 * p1;
    acc = acc + (-1.0) * p2;
    return acc * inv;
}

__device__ __forceinline__ unsigned wrap1(int a, int n) { return (unsigned)(a < 0 ? a + n : (a >= n ? a - n : a)); }

struct RowGroup {
    unsigned x, y0, pl[5], rowy[kRowsY + 4];   // x; first row; planes x-2..x+2; rows y0-2..y0+9 (wrapped)
};

__device__ __forceinline__ RowGroup row_group(Dims d) {
    RowGroup r;
    const unsigned ng = (unsigned)(d.y + kRowsY - 1) / kRowsY;
    r.x = blockIdx.x / ng;
    r.y0 = (blockIdx.x - r.x * ng) * kRowsY;
#pragma unroll
    for (int i = 0; i < 5; ++i) r.pl[i] = wrap1((int)r.x - 2 + i, d.x) * (unsigned)d.y;
#pragma unroll
    for (int i = 0; i < kRowsY + 4; ++i) r.rowy[i] = wrap1((int)r.y0 - 2 + i, d.y);
    return r;
}

__global__ void __launch_bounds__(256) k_grad4_rows(const double* __restrict__ p, Dims d, double h, double scale,
                                                    double* __restrict__ ox, double* __restrict__ oy,
                                                    double* __restrict__ oz) {
    const RowGroup g = row_group(d);
    const double den = 12.0 * h;
    const unsigned nz = (unsigned)d.z;
    for (int z = threadIdx.x; z < d.z; z += blockDim.x) {
        const unsigned zm2 = wrap1(z - 2, d.z), zm1 = wrap1(z - 1, d.z), zp1 = wrap1(z + 1, d.z), zp2 = wrap1(z + 2, d.z);
        double w[kRowsY + 4];
#pragma unroll
        for (int i = 0; i < kRowsY + 4; ++i) w[i] = p[(g.pl[2] + g.rowy[i]) * nz + z];
#pragma unroll
        for (int k = 0; k < kRowsY; ++k) {
            const unsigned y = g.rowy[k + 2];
            const unsigned rc = (g.pl[2] + y) * nz;
            const double gx = g4v(p[(g.pl[0] + y) * nz + z], p[(g.pl[1] + y) * nz + z], p[(g.pl[3] + y) * nz + z],
                                  p[(g.pl[4] + y) * nz + z], den);
            const double gy = g4v(w[k], w[k + 1], w[k + 3], w[k + 4], den);
            const double gz = g4v(p[rc + zm2], p[rc + zm1], p[rc + zp1], p[rc + zp2], den);
            if (g.y0 + k < (unsigned)d.y) {
                ox[rc + z] = scale * gx;
                oy[rc + z] = scale * gy;
                oz[rc + z] = scale * gz;
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_tau_rows(const double* __restrict__ q0, const double* __restrict__ q1,
                                                  const double* __restrict__ q2, Dims d, double h, double post,
                                                  double* __restrict__ tau) {
    const RowGroup g = row_group(d);
    const double den = 12.0 * h;
    const unsigned nz = (unsigned)d.z;
    for (int z = threadIdx.x; z < d.z; z += blockDim.x) {
        const unsigned zm2 = wrap1(z - 2, d.z), zm1 = wrap1(z - 1, d.z), zp1 = wrap1(z + 1, d.z), zp2 = wrap1(z + 2, d.z);
        double w0[kRowsY + 4], w1[kRowsY + 4];
#pragma unroll
        for (int i = 0; i < kRowsY + 4; ++i) {
            w0[i] = q0[(g.pl[2] + g.rowy[i]) * nz + z];
            w1[i] = q1[(g.pl[2] + g.rowy[i]) * nz + z];
        }
#pragma unroll
        for (int k = 0; k < kRowsY; ++k) {
            const unsigned y = g.rowy[k + 2];
            const unsigned rc = (g.pl[2] + y) * nz;
            const double Dxx = g4v(q0[(g.pl[0] + y) * nz + z], q0[(g.pl[1] + y) * nz + z], q0[(g.pl[3] + y) * nz + z],
                                   q0[(g.pl[4] + y) * nz + z], den);
            const double Dyy = g4v(w1[k], w1[k + 1], w1[k + 3], w1[k + 4], den);
            const double Dzz = g4v(q2[rc + zm2], q2[rc + zm1], q2[rc + zp1], q2[rc + zp2], den);
            const double Dyx = g4v(w0[k], w0[k + 1], w0[k + 3], w0[k + 4], den);
            const double Dzx = g4v(q0[rc + zm2], q0[rc + zm1], q0[rc + zp1], q0[rc + zp2], den);
            const double Dzy = g4v(q1[rc + zm2], q1[rc + zm1], q1[rc + zp1], q1[rc + zp2], den);
            double acc = 0.0;
            acc = acc + (Dyy * Dxx - Dyx * Dyx);
            acc = acc + (Dzz * Dxx - Dzx * Dzx);
            acc = acc + (Dzz * Dyy - Dzy * Dzy);
            if (g.y0 + k < (unsigned)d.y) tau[rc + z] = post == 1.0 ? acc : acc * post;
        }
    }
}

// LLA overdensity on a periodic level by groups of rows (the layout of k_grad4_rows): each thread
// takes one z and walks the group's 8 rows; every stencil value is a load at a row base plus z,
// so the per-load index work of the generic kernel (decode, three wraps) is gone.  The same
// operations in the same order as k_lla.
template <bool SUM>
__global__ void __launch_bounds__(256) k_lla_rows(const double* __restrict__ a0, const double* __restrict__ a1,
                                                  const double* __restrict__ a2, const double* __restrict__ b0,
                                                  const double* __restrict__ b1, const double* __restrict__ b2,
                                                  Dims d, double h, double* __restrict__ out) {
    const RowGroup g = row_group(d);
    const double inv = 1.0 / (12.0 * h);
    const unsigned nz = (unsigned)d.z;
    const double* A[3] = {a0, a1, a2};
    const double* Bv[3] = {b0, b1, b2};
    for (int z = threadIdx.x; z < d.z; z += blockDim.x) {
        const unsigned zo[4] = {wrap1(z - 2, d.z), wrap1(z - 1, d.z), wrap1(z + 1, d.z), wrap1(z + 2, d.z)};
        for (int k = 0; k < kRowsY; ++k) {
            if (g.y0 + k >= (unsigned)d.y) break;
            const unsigned y = g.rowy[k + 2];
            const unsigned rc = (g.pl[2] + y) * nz;
            // the four stencil positions along x (planes x-2, x-1, x+1, x+2), y and z
            const unsigned ix[4] = {(g.pl[0] + y) * nz + z, (g.pl[1] + y) * nz + z, (g.pl[3] + y) * nz + z,
                                    (g.pl[4] + y) * nz + z};
            const unsigned iy[4] = {(g.pl[2] + g.rowy[k]) * nz + z, (g.pl[2] + g.rowy[k + 1]) * nz + z,
                                    (g.pl[2] + g.rowy[k + 3]) * nz + z, (g.pl[2] + g.rowy[k + 4]) * nz + z};
            const unsigned iz[4] = {rc + zo[0], rc + zo[1], rc + zo[2], rc + zo[3]};
            double m[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double* ai = A[i];
                const double* bi = Bv[i];
                auto v = [&](unsigned q) {
                    if constexpr (SUM) return ai[q] + bi[q];
                    else return ai[q];
                };
                m[i][0] = 1.0 * (i == 0) + g4m(v(ix[0]), v(ix[1]), v(ix[2]), v(ix[3]), inv);
                m[i][1] = 1.0 * (i == 1) + g4m(v(iy[0]), v(iy[1]), v(iy[2]), v(iy[3]), inv);
                m[i][2] = 1.0 * (i == 2) + g4m(v(iz[0]), v(iz[1]), v(iz[2]), v(iz[3]), inv);
            }
            const double c0 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
            const double c1 = m[1][0] * m[2][2] - m[1][2] * m[2][0];
            const double c2 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
            const double det = (m[0][0] * c0 - m[0][1] * c1) + m[0][2] * c2;
            out[rc + z] = 1.0 / det - 1.0;
        }
    }
}

// ----------------------------------------------------------------------------------------------
// Large periodic levels by tiles marched along x.  A block owns 4 rows x 64 z of 32 consecutive
// planes, one cell per thread and plane.  Each plane's slab (the tile plus 2 cells each side in y
// and z, every component the kernel reads) is loaded into LDS once, into a ring of four slabs:
// the loads of plane x + 3 are issued before plane x is computed and stored into the slot of plane
// x - 1 after it (one barrier per plane).  The y / z stencil values of plane x come from its slab,
// the x-stencil values from a register window of 5 planes filled from the slabs' own cells.
// Consecutive blocks go to the 8 XCDs in turn, so the tiles are renumbered for each XCD to take a
// contiguous run, whose halos are then its own neighbours' cells (in its L2).  Each kernel has
// the same operations in the same order as its row-group version (bit-identical results).
// ----------------------------------------------------------------------------------------------
constexpr int kLtY = 4, kLtZ = 64, kLtX = 32;
constexpr int kSZ = kLtZ + 4, kNS = (kLtY + 4) * kSZ, kPer = (kNS + 255) / 256;

static bool lpt_tiled(Dims d) {
    return d.x % kLtX == 0 && d.y % kLtY == 0 && d.z % kLtZ == 0 && d.cells() >= ((size_t)1 << 21);
}
static unsigned tiles_grid(Dims d) {
    return (unsigned)(d.x / kLtX) * (unsigned)(d.y / kLtY) * (unsigned)(d.z / kLtZ);
}

// Marches the block's tile: val(c, q) is component c at linear index q; NW components (the first
// ones) keep an x-window; plane(x, y, z, slab, me, w) computes and stores the cell (x, y, z) from
// its plane's slab (slab[c][me +- k], me = the cell's slab index) and the windows w[c][0..4]
// (planes x - 2 .. x + 2).
template <int NC, int NW, class V, class F>
__device__ __forceinline__ void march_tiles(Dims d, double (*sl)[NC][kNS], V val, F plane) {
    const unsigned ny = (unsigned)d.y, nz = (unsigned)d.z;
    const unsigned nty = ny / kLtY, ntz = nz / kLtZ;
    unsigned b = blockIdx.x;
    if (gridDim.x % 8 == 0) b = (b % 8) * (gridDim.x / 8) + b / 8;
    const unsigned zt = b % ntz;
    b /= ntz;
    const unsigned yt = b % nty;
    const unsigned x0 = (b / nty) * kLtX;
    const int tz = (int)(threadIdx.x & 63), ty = (int)(threadIdx.x >> 6);
    const unsigned z = zt * kLtZ + tz, y = yt * kLtY + ty;
    const int me = (ty + 2) * kSZ + tz + 2;
    // this thread's share of a slab: entries t = threadIdx.x + 256 r (t < kNS); their in-plane
    // offsets do not depend on the plane (an index past the end is clamped, its value unused)
    unsigned off[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int t = min((int)threadIdx.x + 256 * r, kNS - 1);
        const int sy = t / kSZ, sz = t - sy * kSZ;
        off[r] = wrap1((int)(yt * kLtY) + sy - 2, d.y) * nz + wrap1((int)(zt * kLtZ) + sz - 2, d.z);
    }
    double reg[kPer][NC];
    auto fetch = [&](unsigned xp) {
        const unsigned base = xp * ny * nz;
#pragma unroll
        for (int r = 0; r < kPer; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) reg[r][c] = val(c, base + off[r]);
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int t = (int)threadIdx.x + 256 * r;
            if (t < kNS)
#pragma unroll
                for (int c = 0; c < NC; ++c) sl[slot][c][t] = reg[r][c];
        }
    };
    double w[NW][5];
#pragma unroll
    for (int c = 0; c < NW; ++c) {
        w[c][1] = val(c, (wrap1((int)x0 - 2, d.x) * ny + y) * nz + z);
        w[c][2] = val(c, (wrap1((int)x0 - 1, d.x) * ny + y) * nz + z);
    }
    for (int k = 0; k < 3; ++k) {   // planes x0, x0 + 1, x0 + 2 into slots 0, 1, 2
        fetch(wrap1((int)x0 + k, d.x));
        store(k);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NW; ++c) {
        w[c][3] = sl[0][c][me];
        w[c][4] = sl[1][c][me];
    }
    for (int i = 0; i < kLtX; ++i) {
        const unsigned x = x0 + i;
        const bool more = i + 3 < kLtX + 2;   // the slabs run to plane x0 + kLtX + 1
        if (more) fetch(wrap1((int)x + 3, d.x));
#pragma unroll
        for (int c = 0; c < NW; ++c) {
#pragma unroll
            for (int k = 0; k < 4; ++k) w[c][k] = w[c][k + 1];
            w[c][4] = sl[(i + 2) & 3][c][me];
        }
        plane(x, y, z, sl[i & 3], me, w);
        // slot (i + 3) & 3 held plane x - 1, last read in iteration i - 1 (before the previous
        // barrier); plane x + 3 goes there and is read after this barrier
        if (more) store((i + 3) & 3);
        __syncthreads();
    }
}

// LLA overdensity (as k_lla_rows)
template <bool SUM>
__global__ void __launch_bounds__(256) k_lla_tile(const double* __restrict__ a0, const double* __restrict__ a1,
                                                  const double* __restrict__ a2, const double* __restrict__ b0,
                                                  const double* __restrict__ b1, const double* __restrict__ b2,
                                                  Dims d, double h, double* __restrict__ out) {
    __shared__ double sl[4][3][kNS];
    const double* A[3] = {a0, a1, a2};
    const double* Bv[3] = {b0, b1, b2};
    const double inv = 1.0 / (12.0 * h);
    const unsigned ny = (unsigned)d.y, nz = (unsigned)d.z;
    auto val = [&](int c, unsigned q) {
        if constexpr (SUM) return A[c][q] + Bv[c][q];
        else return A[c][q];
    };
    march_tiles<3, 3>(d, sl, val, [&](unsigned x, unsigned y, unsigned z, double (*s)[kNS], int me, double (*w)[5]) {
        double m[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            m[c][0] = 1.0 * (c == 0) + g4m(w[c][0], w[c][1], w[c][3], w[c][4], inv);
            m[c][1] = 1.0 * (c == 1) + g4m(s[c][me - 2 * kSZ], s[c][me - kSZ], s[c][me + kSZ], s[c][me + 2 * kSZ], inv);
            m[c][2] = 1.0 * (c == 2) + g4m(s[c][me - 2], s[c][me - 1], s[c][me + 1], s[c][me + 2], inv);
        }
        const double c0 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
        const double c1 = m[1][0] * m[2][2] - m[1][2] * m[2][0];
        const double c2 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
        const double det = (m[0][0] * c0 - m[0][1] * c1) + m[0][2] * c2;
        out[(x * ny + y) * nz + z] = 1.0 / det - 1.0;
    });
}

// psi_c = scale * G4_c phi (as k_grad4_rows)
__global__ void __launch_bounds__(256) k_grad4_tile(const double* __restrict__ p, Dims d, double h, double scale,
                                                    double* __restrict__ ox, double* __restrict__ oy,
                                                    double* __restrict__ oz) {
    __shared__ double sl[4][1][kNS];
    const double den = 12.0 * h;
    const unsigned ny = (unsigned)d.y, nz = (unsigned)d.z;
    march_tiles<1, 1>(d, sl, [&](int, unsigned q) { return p[q]; },
                      [&](unsigned x, unsigned y, unsigned z, double (*s)[kNS], int me, double (*w)[5]) {
                          const double gx = g4v(w[0][0], w[0][1], w[0][3], w[0][4], den);
                          const double gy = g4v(s[0][me - 2 * kSZ], s[0][me - kSZ], s[0][me + kSZ], s[0][me + 2 * kSZ], den);
                          const double gz = g4v(s[0][me - 2], s[0][me - 1], s[0][me + 1], s[0][me + 2], den);
                          const unsigned q = (x * ny + y) * nz + z;
                          ox[q] = scale * gx;
                          oy[q] = scale * gy;
                          oz[q] = scale * gz;
                      });
}

// tau from the three gradient components (as k_tau_rows)
__global__ void __launch_bounds__(256) k_tau_tile(const double* __restrict__ q0, const double* __restrict__ q1,
                                                  const double* __restrict__ q2, Dims d, double h, double post,
                                                  double* __restrict__ tau) {
    __shared__ double sl[4][3][kNS];
    const double* Q[3] = {q0, q1, q2};
    const double den = 12.0 * h;
    const unsigned ny = (unsigned)d.y, nz = (unsigned)d.z;
    march_tiles<3, 1>(d, sl, [&](int c, unsigned q) { return Q[c][q]; },
                      [&](unsigned x, unsigned y, unsigned z, double (*s)[kNS], int me, double (*w)[5]) {
                          const double Dxx = g4v(w[0][0], w[0][1], w[0][3], w[0][4], den);
                          const double Dyy = g4v(s[1][me - 2 * kSZ], s[1][me - kSZ], s[1][me + kSZ], s[1][me + 2 * kSZ], den);
                          const double Dzz = g4v(s[2][me - 2], s[2][me - 1], s[2][me + 1], s[2][me + 2], den);
                          const double Dyx = g4v(s[0][me - 2 * kSZ], s[0][me - kSZ], s[0][me + kSZ], s[0][me + 2 * kSZ], den);
                          const double Dzx = g4v(s[0][me - 2], s[0][me - 1], s[0][me + 1], s[0][me + 2], den);
                          const double Dzy = g4v(s[1][me - 2], s[1][me - 1], s[1][me + 1], s[1][me + 2], den);
                          double acc = 0.0;
                          acc = acc + (Dyy * Dxx - Dyx * Dyx);
                          acc = acc + (Dzz * Dxx - Dzx * Dzx);
                          acc = acc + (Dzz * Dyy - Dzy * Dzy);
                          tau[(x * ny + y) * nz + z] = post == 1.0 ? acc : acc * post;
                      });
}


static unsigned rows_grid(Dims d) { return (unsigned)d.x * (unsigned)((d.y + kRowsY - 1) / kRowsY); }
static unsigned rows_block(Dims d) { return d.z >= 256 ? 256u : (unsigned)((d.z + 63) / 64 * 64); }

// padded copy of a patch with width-R tri-quadratic ghosts from its parent
__global__ void k_wide_ghost(const double* __restrict__ pu, const double* __restrict__ u, double* __restrict__ out,
                             Dims d, ParentMap pm, int R, Lay B) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int gx, gy, gz;
    decode3(B, t, gx, gy, gz);
    const int i[3] = {gx - R, gy - R, gz - R};
    const int n[3] = {d.x, d.y, d.z};
    if (i[0] >= 0 && i[0] < n[0] && i[1] >= 0 && i[1] < n[1] && i[2] >= 0 && i[2] < n[2]) {
        out[t] = u[((size_t)i[0] * d.y + i[1]) * d.z + i[2]];
        return;
    }
    int P[3];
    double w[3][3];
    for (int a = 0; a < 3; ++a) {
        P[a] = pm.off[a] + (i[a] >> 1);       // floor division, also for negative i
        const double tt = (i[a] & 1) ? 0.25 : -0.25;
        w[a][0] = 0.5 * tt * (tt - 1.0);
        w[a][1] = 1.0 - tt * tt;
        w[a][2] = 0.5 * tt * (tt + 1.0);
    }
    const int pdim[3] = {pm.pl.d.x, pm.pl.d.y, pm.pl.d.z};
    // interpolate along x, then y, then z (tensor product)
    double az = 0.0;
    for (int dz = 0; dz < 3; ++dz) {
        double ay = 0.0;
        for (int dy = 0; dy < 3; ++dy) {
            double ax = 0.0;
            for (int dx = 0; dx < 3; ++dx) {
                int q[3] = {P[0] + dx - 1, P[1] + dy - 1, P[2] + dz - 1};
                if (pm.periodic)
                    for (int k = 0; k < 3; ++k) q[k] = q[k] < 0 ? q[k] + pdim[k] : (q[k] >= pdim[k] ? q[k] - pdim[k] : q[k]);
                ax = ax + w[0][dx] * pu[((size_t)q[0] * pdim[1] + q[1]) * pdim[2] + q[2]];
            }
            ay = ay + w[1][dy] * ax;
        }
        az = az + w[2][dz] * ay;
    }
    out[t] = az;
}

void launch_wide_ghost(const double* pu, const double* u, double* padded, Dims d, ParentMap pm, int R,
                       hipStream_t st) {
    const Lay B(Dims{d.x + 2 * R, d.y + 2 * R, d.z + 2 * R}, 0);
    k_wide_ghost<<<grid_for(B.d.cells()), kBlock, 0, st>>>(pu, u, padded, d, pm, R, B);
}

void launch_grad4(const double* src, int R, Dims d, double h, double scale, double* ox, double* oy, double* oz,
                  hipStream_t st, int order) {
    const Lay B(d, 0);
    if (order == 6) {   // the sixth-order gradient: one thread per cell (periodic, or padded by R >= 3)
        if (R == 0)
            k_grad4<false, 6><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<false>{src, 0, d}, B, h, scale, ox, oy, oz);
        else
            k_grad4<true, 6><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<true>{src, R, d}, B, h, scale, ox, oy, oz);
        return;
    }
    if (R == 0 && lpt_tiled(d))
        k_grad4_tile<<<tiles_grid(d), 256, 0, st>>>(src, d, h, scale, ox, oy, oz);
    else if (R == 0)
        k_grad4_rows<<<rows_grid(d), rows_block(d), 0, st>>>(src, d, h, scale, ox, oy, oz);
    else
        k_grad4<true><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<true>{src, R, d}, B, h, scale, ox, oy, oz);
}

void launch_tau(const double* src, int R, Dims d, double h, double* tau, double* psi, hipStream_t st, int order) {
    const int rg = order / 2;   // the gradient's radius
    const int e = R >= rg ? R - rg : 0;
    const Lay E(Dims{d.x + 2 * e, d.y + 2 * e, d.z + 2 * e}, 0);
    const Lay B(d, 0);
    double* p0 = psi;
    double* p1 = psi + E.d.cells();
    double* p2 = psi + 2 * E.d.cells();
    if (order == 6) {   // the sixth-order gradient twice: one thread per cell
        if (R == 0) {
            k_psi<false, 6><<<grid_for(E.d.cells()), kBlock, 0, st>>>(Src<false>{src, 0, d}, E, 0, h, p0, p1, p2);
            k_tau_psi<false, 6><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<false>{p0, 0, d}, Src<false>{p1, 0, d},
                                                                        Src<false>{p2, 0, d}, B, h, 1.0, tau);
        } else {
            k_psi<true, 6><<<grid_for(E.d.cells()), kBlock, 0, st>>>(Src<true>{src, R, d}, E, e, h, p0, p1, p2);
            k_tau_psi<true, 6><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<true>{p0, e, d}, Src<true>{p1, e, d},
                                                                       Src<true>{p2, e, d}, B, h, 1.0, tau);
        }
        return;
    }
    if (R == 0) {
        k_psi<false><<<grid_for(E.d.cells()), kBlock, 0, st>>>(Src<false>{src, 0, d}, E, 0, h, p0, p1, p2);
        if (lpt_tiled(d)) k_tau_tile<<<tiles_grid(d), 256, 0, st>>>(p0, p1, p2, d, h, 1.0, tau);
        else k_tau_rows<<<rows_grid(d), rows_block(d), 0, st>>>(p0, p1, p2, d, h, 1.0, tau);
    } else {
        k_psi<true><<<grid_for(E.d.cells()), kBlock, 0, st>>>(Src<true>{src, R, d}, E, e, h, p0, p1, p2);
        k_tau_psi<true><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<true>{p0, e, d}, Src<true>{p1, e, d},
                                                                Src<true>{p2, e, d}, B, h, 1.0, tau);
    }
}

void launch_tau_from_grad(const double* g0, const double* g1, const double* g2, Dims d, double h, double post,
                         double* tau, hipStream_t st, int order) {
    if (order == 6) {
        k_tau_psi<false, 6><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<false>{g0, 0, d}, Src<false>{g1, 0, d},
                                                                    Src<false>{g2, 0, d}, Lay(d, 0), h, post, tau);
        return;
    }
    if (lpt_tiled(d)) k_tau_tile<<<tiles_grid(d), 256, 0, st>>>(g0, g1, g2, d, h, post, tau);
    else k_tau_rows<<<rows_grid(d), rows_block(d), 0, st>>>(g0, g1, g2, d, h, post, tau);
}


void launch_lla(const double* const* a, const double* const* b, int R, Dims d, double h, double* out, hipStream_t st) {
    const Lay B(d, 0);
    const int sum = b != nullptr;
    const double* const* bb = sum ? b : a;
    // periodic levels (every base here has at least 2 cells per axis, so a single wrap of an
    // offset of 2 holds) by x-marched tiles where they divide the level, else by groups of rows;
    // padded patches by the per-cell kernel
    if (R == 0 && lpt_tiled(d)) {
        if (sum) k_lla_tile<true><<<tiles_grid(d), 256, 0, st>>>(a[0], a[1], a[2], bb[0], bb[1], bb[2], d, h, out);
        else k_lla_tile<false><<<tiles_grid(d), 256, 0, st>>>(a[0], a[1], a[2], bb[0], bb[1], bb[2], d, h, out);
    } else if (R == 0 && sum)
        k_lla_rows<true><<<rows_grid(d), rows_block(d), 0, st>>>(a[0], a[1], a[2], bb[0], bb[1], bb[2], d, h, out);
    else if (R == 0)
        k_lla_rows<false><<<rows_grid(d), rows_block(d), 0, st>>>(a[0], a[1], a[2], bb[0], bb[1], bb[2], d, h, out);
    else
        k_lla<true><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<true>{a[0], R, d}, Src<true>{a[1], R, d},
                                                           Src<true>{a[2], R, d}, Src<true>{bb[0], R, d},
                                                           Src<true>{bb[1], R, d}, Src<true>{bb[2], R, d}, sum, B, h,
                                                           out);
}

void launch_add2(const double* a, const double* b, double* dst, size_t n, hipStream_t st) {
    k_add2<<<grid_for(n), kBlock, 0, st>>>(a, b, dst, n);
}

}  // namespace mgic
