// LPT kernels for gfx950 (Hahn & Abel 2011, Section 3.1):
//   first order   psi_c = scale * G4_c phi           (Table 1 fourth-order gradient)
//   second order  tau = sum_{i>j} D_ii D_jj - D_ij^2,  D_ij = G4_i (G4_j phi)
// plus the post-solve ghost layers of width R (faces, edges and corners) that patches need:
// coarse-only tri-quadratic interpolation of the parent at the child's position (children sit at
// -1/4 and +1/4 of the parent cell along each axis).
//
// Sources are either periodic n^3 arrays (R = 0: indices wrap) or arrays padded by R ghost cells
// on every side.  The gradient is evaluated as ((u[-2] - 8 u[-1]) + 8 u[+1]) - u[+2], / (12 h),
// then scaled.  tau takes two passes: psi_j = G4_j phi is stored (extended by 2 cells on
// patches), then D_ij = G4_i psi_j is evaluated per cell.

#include "mg_internal.h"

namespace mgic {

struct Src {
    const double* p;
    int R;       // 0: periodic wrap over d; > 0: padded by R
    Dims d;      // interior dims
    __device__ __forceinline__ double at(int x, int y, int z) const {
        if (R == 0) {
            x = x < 0 ? x + d.x : (x >= d.x ? x - d.x : x);
            y = y < 0 ? y + d.y : (y >= d.y ? y - d.y : y);
            z = z < 0 ? z + d.z : (z >= d.z ? z - d.z : z);
            return p[((size_t)x * d.y + y) * d.z + z];
        }
        const size_t py = (size_t)d.y + 2 * R, pz = (size_t)d.z + 2 * R;
        return p[((size_t)(x + R) * py + (y + R)) * pz + (z + R)];
    }
};

// fourth-order gradient of s along `axis` at (x, y, z), Table 1 weights (1, -8, 0, 8, -1) / 12
__device__ __forceinline__ double g4(const Src& s, int x, int y, int z, int axis, double den) {
    const int ex = axis == 0, ey = axis == 1, ez = axis == 2;
    double acc = s.at(x - 2 * ex, y - 2 * ey, z - 2 * ez);
    acc = acc + (-8.0) * s.at(x - ex, y - ey, z - ez);
    acc = acc + 8.0 * s.at(x + ex, y + ey, z + ez);
    acc = acc + (-1.0) * s.at(x + 2 * ex, y + 2 * ey, z + 2 * ez);
    return acc / den;
}

__global__ void k_grad4(Src s, double h, double scale, double* __restrict__ ox, double* __restrict__ oy,
                        double* __restrict__ oz) {
    const Dims d = s.d;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= d.cells()) return;
    const int z = (int)(t % d.z);
    const int y = (int)((t / d.z) % d.y);
    const int x = (int)(t / ((size_t)d.z * d.y));
    const double den = 12.0 * h;
    ox[t] = scale * g4(s, x, y, z, 0, den);
    oy[t] = scale * g4(s, x, y, z, 1, den);
    oz[t] = scale * g4(s, x, y, z, 2, den);
}

// psi_j = G4_j phi on the interior extended by e cells (e <= R - 2), unscaled; output arrays
// are (d + 2e)^3, padded by e
__global__ void k_psi(Src s, int e, double h, double* __restrict__ p0, double* __restrict__ p1,
                      double* __restrict__ p2) {
    const Dims od{s.d.x + 2 * e, s.d.y + 2 * e, s.d.z + 2 * e};
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= od.cells()) return;
    const int z = (int)(t % od.z) - e;
    const int y = (int)((t / od.z) % od.y) - e;
    const int x = (int)(t / ((size_t)od.z * od.y)) - e;
    const double den = 12.0 * h;
    p0[t] = g4(s, x, y, z, 0, den);
    p1[t] = g4(s, x, y, z, 1, den);
    p2[t] = g4(s, x, y, z, 2, den);
}

// tau = sum_{i>j} D_ii D_jj - D_ij^2 with D_ij = G4_i psi_j; psi periodic (e = 0) or padded by e
__global__ void k_tau_psi(Src q0, Src q1, Src q2, double h, double* __restrict__ tau) {
    const Dims d = q0.d;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= d.cells()) return;
    const int z = (int)(t % d.z);
    const int y = (int)((t / d.z) % d.y);
    const int x = (int)(t / ((size_t)d.z * d.y));
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
    tau[t] = acc;
}

// padded copy of a patch with width-R tri-quadratic ghosts from its parent
__global__ void k_wide_ghost(const double* __restrict__ pu, const double* __restrict__ u, double* __restrict__ out,
                             Dims d, ParentMap pm, int R) {
    const Dims pd{d.x + 2 * R, d.y + 2 * R, d.z + 2 * R};
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= pd.cells()) return;
    const int gz = (int)(t % pd.z);
    const int gy = (int)((t / pd.z) % pd.y);
    const int gx = (int)(t / ((size_t)pd.z * pd.y));
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
    const int pdim[3] = {pm.pd.x, pm.pd.y, pm.pd.z};
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
    const size_t n = (size_t)(d.x + 2 * R) * (d.y + 2 * R) * (d.z + 2 * R);
    k_wide_ghost<<<grid_for(n), kBlock, 0, st>>>(pu, u, padded, d, pm, R);
}

void launch_grad4(const double* src, int R, Dims d, double h, double scale, double* ox, double* oy, double* oz,
                  hipStream_t st) {
    k_grad4<<<grid_for(d.cells()), kBlock, 0, st>>>(Src{src, R, d}, h, scale, ox, oy, oz);
}

void launch_tau(const double* src, int R, Dims d, double h, double* tau, double* psi, hipStream_t st) {
    const int e = R >= 2 ? R - 2 : 0;
    const Dims od{d.x + 2 * e, d.y + 2 * e, d.z + 2 * e};
    double* p0 = psi;
    double* p1 = psi + od.cells();
    double* p2 = psi + 2 * od.cells();
    k_psi<<<grid_for(od.cells()), kBlock, 0, st>>>(Src{src, R, d}, e, h, p0, p1, p2);
    k_tau_psi<<<grid_for(d.cells()), kBlock, 0, st>>>(Src{p0, e, d}, Src{p1, e, d}, Src{p2, e, d}, h, tau);
}

}  // namespace mgic
