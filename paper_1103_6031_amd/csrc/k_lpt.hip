// LPT kernels for gfx950 (Hahn & Abel 2011, Section 3.1):
//   first order   psi_c = scale * G4_c phi           (Table 1 fourth-order gradient)
//   second order  tau = sum_{i>j} D_ii D_jj - D_ij^2,  D_ij = G4_i (G4_j phi)
// plus the post-solve ghost layers of width R (faces, edges and corners) that patches need:
// coarse-only tri-quadratic interpolation of the parent at the child's position (children sit at
// -1/4 and +1/4 of the parent cell along each axis).
//
// Sources are either periodic n^3 arrays (indices wrap) or arrays padded by R ghost cells on
// every side; the two cases are separate instantiations.  The gradient is evaluated as
// ((u[-2] - 8 u[-1]) + 8 u[+1]) - u[+2], / (12 h), then scaled.  tau takes two passes:
// psi_j = G4_j phi is stored (extended by 2 cells on patches), then D_ij = G4_i psi_j is
// evaluated per cell.  Output cells are decoded from a linear index with multiply-shift
// division (every array has fewer than 2^31 cells).

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

// linear index -> (x, y, z) of a box, natural order
__device__ __forceinline__ void decode3(const Lay& B, unsigned t, int& x, int& y, int& z) {
    const unsigned row = B.dz.div(t);
    z = (int)(t - row * (unsigned)B.d.z);
    const unsigned xq = B.dy.div(row);
    y = (int)(row - xq * (unsigned)B.d.y);
    x = (int)xq;
}

template <bool PAD>
__global__ void k_grad4(Src<PAD> s, Lay B, double h, double scale, double* __restrict__ ox,
                        double* __restrict__ oy, double* __restrict__ oz) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int x, y, z;
    decode3(B, t, x, y, z);
    const double den = 12.0 * h;
    ox[t] = scale * g4(s, x, y, z, 0, den);
    oy[t] = scale * g4(s, x, y, z, 1, den);
    oz[t] = scale * g4(s, x, y, z, 2, den);
}

// psi_j = G4_j phi on the interior extended by e cells (e <= R - 2), unscaled; the output box B
// is (d + 2e)^3, padded by e
template <bool PAD>
__global__ void k_psi(Src<PAD> s, Lay B, int e, double h, double* __restrict__ p0, double* __restrict__ p1,
                      double* __restrict__ p2) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int x, y, z;
    decode3(B, t, x, y, z);
    x -= e;
    y -= e;
    z -= e;
    const double den = 12.0 * h;
    p0[t] = g4(s, x, y, z, 0, den);
    p1[t] = g4(s, x, y, z, 1, den);
    p2[t] = g4(s, x, y, z, 2, den);
}

// tau = sum_{i>j} D_ii D_jj - D_ij^2 with D_ij = G4_i psi_j; psi periodic or padded by e.  When
// psi is a scaled gradient s G4 phi, post = 1 / s^2 brings tau back to the one of phi (post = 1:
// not applied, so s = +-1 gives the same bits as psi = G4 phi)
template <bool PAD>
__global__ void k_tau_psi(Src<PAD> q0, Src<PAD> q1, Src<PAD> q2, Lay B, double h, double post,
                          double* __restrict__ tau) {
    const unsigned t = (unsigned)lpt_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)B.d.cells()) return;
    int x, y, z;
    decode3(B, t, x, y, z);
    const double den = 12.0 * h;
    const double Dxx = g4(q0, x, y, z, 0, den);
    const double Dyy = g4(q1, x, y, z, 1, den);
    const double Dzz = g4(q2, x, y, z, 2, den);
    const double Dyx = g4(q0, x, y, z, 1, den);
    const double Dzx = g4(q0, x, y, z, 2, den);
    const double Dzy = g4(q1, x, y, z, 2, den);
    double acc = 0.0;
    acc = acc + (Dyy * Dxx - Dyx * Dyx);
    acc = acc + (Dzz * Dxx - Dzx * Dzx);
    acc = acc + (Dzz * Dyy - Dzy * Dzy);
    tau[t] = post == 1.0 ? acc : acc * post;
}

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
                  hipStream_t st) {
    const Lay B(d, 0);
    if (R == 0)
        k_grad4<false><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<false>{src, 0, d}, B, h, scale, ox, oy, oz);
    else
        k_grad4<true><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<true>{src, R, d}, B, h, scale, ox, oy, oz);
}

void launch_tau(const double* src, int R, Dims d, double h, double* tau, double* psi, hipStream_t st) {
    const int e = R >= 2 ? R - 2 : 0;
    const Lay E(Dims{d.x + 2 * e, d.y + 2 * e, d.z + 2 * e}, 0);
    const Lay B(d, 0);
    double* p0 = psi;
    double* p1 = psi + E.d.cells();
    double* p2 = psi + 2 * E.d.cells();
    if (R == 0) {
        k_psi<false><<<grid_for(E.d.cells()), kBlock, 0, st>>>(Src<false>{src, 0, d}, E, 0, h, p0, p1, p2);
        k_tau_psi<false><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<false>{p0, 0, d}, Src<false>{p1, 0, d},
                                                                 Src<false>{p2, 0, d}, B, h, 1.0, tau);
    } else {
        k_psi<true><<<grid_for(E.d.cells()), kBlock, 0, st>>>(Src<true>{src, R, d}, E, e, h, p0, p1, p2);
        k_tau_psi<true><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<true>{p0, e, d}, Src<true>{p1, e, d},
                                                                Src<true>{p2, e, d}, B, h, 1.0, tau);
    }
}

void launch_tau_from_grad(const double* g0, const double* g1, const double* g2, Dims d, double h, double post,
                         double* tau, hipStream_t st) {
    const Lay B(d, 0);
    k_tau_psi<false><<<grid_for(d.cells()), kBlock, 0, st>>>(Src<false>{g0, 0, d}, Src<false>{g1, 0, d},
                                                             Src<false>{g2, 0, d}, B, h, post, tau);
}

}  // namespace mgic
