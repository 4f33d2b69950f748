// Multi-scale density on nested grids (Sections 2.1-2.3 and 3.5.3 of Hahn & Abel 2011): kernel
// grids per level, the grid work of the noise refinement and of the nested convolutions.  The
// transforms themselves are the passes of k_fft.hip, driven from density.cpp.
//
// Arrays are natural [x][y][z] with z contiguous.  Kernel grids are FFT grids: index j of an axis
// of P points is the displacement j (j < P/2) or j - P cells.  A patch's padded domain D' has 2n
// cells per axis and holds the patch itself at [n/2, 3n/2).

#include "spec_internal.h"

namespace mgic {

namespace {

__device__ __forceinline__ int fft_disp(int j, int P) { return j < P / 2 ? j : j - P; }

// T(r) by linear interpolation of table[i] = T(i dr)
__device__ __forceinline__ double radial_at(const double* __restrict__ table, double dr, double r) {
    const double t = r / dr;
    const double fl = floor(t);
    const long long i = (long long)fl;
    const double w = t - fl;
    return (1.0 - w) * table[i] + w * table[i + 1];
}

__device__ __forceinline__ void unflat(size_t idx, int n1, int n2, int& x, int& y, int& z) {
    z = (int)(idx % (size_t)n2);
    const size_t r = idx / (size_t)n2;
    y = (int)(r % (size_t)n1);
    x = (int)(r / (size_t)n1);
}

// T on the displacement grid (Section 2.2), or the mean over the 8 sub-cell centres (Section 3.5.3)
__global__ void k_kernel_direct(double* __restrict__ T, int p0, int p1, int p2, double h,
                                const double* __restrict__ table, double dr, int subgrid) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)p0 * p1 * p2) return;
    int x, y, z;
    unflat(idx, p1, p2, x, y, z);
    const double dx = (double)fft_disp(x, p0) * h, dy = (double)fft_disp(y, p1) * h, dz = (double)fft_disp(z, p2) * h;
    if (!subgrid) {
        T[idx] = radial_at(table, dr, sqrt(dx * dx + dy * dy + dz * dz));
        return;
    }
    double acc = 0.0;
    for (int sx = 0; sx < 2; ++sx)
        for (int sy = 0; sy < 2; ++sy)
            for (int sz = 0; sz < 2; ++sz) {
                const double X = dx + (sx ? 0.25 : -0.25) * h, Y = dy + (sy ? 0.25 : -0.25) * h,
                             Z = dz + (sz ? 0.25 : -0.25) * h;
                acc = acc + radial_at(table, dr, sqrt(X * X + Y * Y + Z * Z));
            }
    T[idx] = acc / 8.0;
}

// T is even in each displacement component (a radial function; the sub-cell centres and the
// child-pair weights are symmetric), so on a grid with even extents one octant of displacements
// c in [0, P/2] per axis is evaluated and written to its mirror images: index c and, for
// 0 < c < P/2, index P - c (index P/2 holds -P/2, whose value is that of +P/2).  An eighth of the
// evaluations, the same values up to the order of the sums.
__device__ __forceinline__ void write_mirrors(double* __restrict__ T, int p0, int p1, int p2, int cx, int cy, int cz,
                                              double v) {
    const int xs[2] = {cx, p0 - cx}, ys[2] = {cy, p1 - cy}, zs[2] = {cz, p2 - cz};
    const int nx = (cx > 0 && 2 * cx != p0) ? 2 : 1, ny = (cy > 0 && 2 * cy != p1) ? 2 : 1,
              nz = (cz > 0 && 2 * cz != p2) ? 2 : 1;
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < ny; ++b)
            for (int c = 0; c < nz; ++c) T[((size_t)xs[a] * p1 + ys[b]) * p2 + zs[c]] = v;
}

__global__ void k_kernel_direct_oct(double* __restrict__ T, int p0, int p1, int p2, double h,
                                    const double* __restrict__ table, double dr, int subgrid) {
    const int q1 = p1 / 2 + 1, q2 = p2 / 2 + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)(p0 / 2 + 1) * q1 * q2) return;
    int cx, cy, cz;
    unflat(idx, q1, q2, cx, cy, cz);
    const double dx = (double)cx * h, dy = (double)cy * h, dz = (double)cz * h;
    double v;
    if (!subgrid) {
        v = radial_at(table, dr, sqrt(dx * dx + dy * dy + dz * dz));
    } else {
        double acc = 0.0;
        for (int sx = 0; sx < 2; ++sx)
            for (int sy = 0; sy < 2; ++sy)
                for (int sz = 0; sz < 2; ++sz) {
                    const double X = dx + (sx ? 0.25 : -0.25) * h, Y = dy + (sy ? 0.25 : -0.25) * h,
                                 Z = dz + (sz ? 0.25 : -0.25) * h;
                    acc = acc + radial_at(table, dr, sqrt(X * X + Y * Y + Z * Z));
                }
        v = acc / 8.0;
    }
    write_mirrors(T, p0, p1, p2, cx, cy, cz, v);
}

// coarse kernel from the finer level's grid: the 1/4, 1/2, 1/4 child-pair mean over the fine
// displacements 2J - 1, 2J, 2J + 1 where all exist (|J| <= Pf / 4 - 1 per axis), T(|D|) elsewhere
__global__ void k_kernel_restrict(double* __restrict__ Tc, int p0, int p1, int p2, double h,
                                  const double* __restrict__ Tf, int f0, int f1, int f2,
                                  const double* __restrict__ table, double dr) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)p0 * p1 * p2) return;
    int x, y, z;
    unflat(idx, p1, p2, x, y, z);
    const int Jx = fft_disp(x, p0), Jy = fft_disp(y, p1), Jz = fft_disp(z, p2);
    const bool inside = abs(Jx) <= f0 / 4 - 1 && abs(Jy) <= f1 / 4 - 1 && abs(Jz) <= f2 / 4 - 1;
    if (!inside) {
        const double dx = (double)Jx * h, dy = (double)Jy * h, dz = (double)Jz * h;
        Tc[idx] = radial_at(table, dr, sqrt(dx * dx + dy * dy + dz * dz));
        return;
    }
    const double w[3] = {0.25, 0.5, 0.25};
    double acc = 0.0;
    for (int sx = -1; sx <= 1; ++sx) {
        const int ix = (2 * Jx + sx + f0) % f0;
        for (int sy = -1; sy <= 1; ++sy) {
            const int iy = (2 * Jy + sy + f1) % f1;
            for (int sz = -1; sz <= 1; ++sz) {
                const int iz = (2 * Jz + sz + f2) % f2;
                acc = acc + ((w[sx + 1] * w[sy + 1]) * w[sz + 1]) * Tf[((size_t)ix * f1 + iy) * f2 + iz];
            }
        }
    }
    Tc[idx] = acc;
}

// k_kernel_restrict on one octant (even extents), written to the mirror images
__global__ void k_kernel_restrict_oct(double* __restrict__ Tc, int p0, int p1, int p2, double h,
                                      const double* __restrict__ Tf, int f0, int f1, int f2,
                                      const double* __restrict__ table, double dr) {
    const int q1 = p1 / 2 + 1, q2 = p2 / 2 + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)(p0 / 2 + 1) * q1 * q2) return;
    int Jx, Jy, Jz;
    unflat(idx, q1, q2, Jx, Jy, Jz);
    const bool inside = Jx <= f0 / 4 - 1 && Jy <= f1 / 4 - 1 && Jz <= f2 / 4 - 1;
    double v;
    if (!inside) {
        const double dx = (double)Jx * h, dy = (double)Jy * h, dz = (double)Jz * h;
        v = radial_at(table, dr, sqrt(dx * dx + dy * dy + dz * dz));
    } else {
        const double w[3] = {0.25, 0.5, 0.25};
        double acc = 0.0;
        for (int sx = -1; sx <= 1; ++sx) {
            const int ix = (2 * Jx + sx + f0) % f0;
            for (int sy = -1; sy <= 1; ++sy) {
                const int iy = (2 * Jy + sy + f1) % f1;
                for (int sz = -1; sz <= 1; ++sz) {
                    const int iz = (2 * Jz + sz + f2) % f2;
                    acc = acc + ((w[sx + 1] * w[sy + 1]) * w[sz + 1]) * Tf[((size_t)ix * f1 + iy) * f2 + iz];
                }
            }
        }
        v = acc;
    }
    write_mirrors(Tc, p0, p1, p2, Jx, Jy, Jz, v);
}

__global__ void k_divide(double* __restrict__ out, const double* __restrict__ in, size_t n, double d) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] / d;
}

// a box of n[] cells of a parent array (dims pd[], box start po[] + lo[], wrapping by wrap > 0)
struct Box {
    int pd[3];   // parent array dims
    int po[3];   // where the parent's own cells start inside its array
    int lo[3];   // box start in the parent's own cells
    int wrap;    // the parent is periodic with this many cells per axis (0: no wrap)
};
__device__ __forceinline__ size_t box_at(const Box& B, int i, int j, int k) {
    int x = B.lo[0] + i, y = B.lo[1] + j, z = B.lo[2] + k;
    if (B.wrap) {
        x = ((x % B.wrap) + B.wrap) % B.wrap;
        y = ((y % B.wrap) + B.wrap) % B.wrap;
        z = ((z % B.wrap) + B.wrap) % B.wrap;
    }
    return ((size_t)(B.po[0] + x) * B.pd[1] + (B.po[1] + y)) * B.pd[2] + (B.po[2] + z);
}

__global__ void k_gather(double* __restrict__ dst, int n0, int n1, int n2, const double* __restrict__ src, Box B) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n0 * n1 * n2) return;
    int x, y, z;
    unflat(idx, n1, n2, x, y, z);
    dst[idx] = src[box_at(B, x, y, z)];
}

// parent box cell I := mean of the 8 children at child array position co + 2I (child dims cd)
__global__ void k_restrict_mean(double* __restrict__ parent, Box B, int m0, int m1, int m2,
                                const double* __restrict__ child, int c0, int c1, int c2, int cox, int coy,
                                int coz) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)m0 * m1 * m2) return;
    int x, y, z;
    unflat(idx, m1, m2, x, y, z);
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                s = s + child[((size_t)(cox + 2 * x + a) * c1 + (coy + 2 * y + b)) * c2 + (coz + 2 * z + c)];
    parent[box_at(B, x, y, z)] = s / 8.0;
}

// base noise with the cells of the first patch zeroed
__global__ void k_zero_box(double* __restrict__ out, const double* __restrict__ in, int n0, int n1, int n2, int lx,
                           int ly, int lz, int mx, int my, int mz) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n0 * n1 * n2) return;
    int x, y, z;
    unflat(idx, n1, n2, x, y, z);
    const bool cov = x >= lx && x < lx + mx && y >= ly && y < ly + my && z >= lz && z < lz + mz;
    out[idx] = cov ? 0.0 : in[idx];
}

// the inputs of a patch level's convolutions on D' (2n per axis):
//   a = the noise inside the patch, noise minus its parent's value on the padding
//   b = 0 inside the patch, noise minus its parent's value on the padding
//   c = the noise inside the patch except the next patch's covered cells, 0 on the padding
__global__ void k_conv_prep(double* __restrict__ a, double* __restrict__ b, double* __restrict__ c,
                            const double* __restrict__ mu, int n0, int n1, int n2, const double* __restrict__ par,
                            Box B, int nx0, int ny0, int nz0, int nmx, int nmy, int nmz) {
    const int d0 = 2 * n0, d1 = 2 * n1, d2 = 2 * n2;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)d0 * d1 * d2) return;
    int x, y, z;
    unflat(idx, d1, d2, x, y, z);
    const bool inside = x >= n0 / 2 && x < n0 / 2 + n0 && y >= n1 / 2 && y < n1 / 2 + n1 && z >= n2 / 2 &&
                        z < n2 / 2 + n2;
    const double m = mu[idx];
    if (inside) {
        a[idx] = m;
        b[idx] = 0.0;
    } else {
        const double d = m - par[box_at(B, x >> 1, y >> 1, z >> 1)];
        a[idx] = d;
        b[idx] = d;
    }
    if (c) {
        const int px = x - n0 / 2, py = y - n1 / 2, pz = z - n2 / 2;
        const bool nxt = px >= nx0 && px < nx0 + nmx && py >= ny0 && py < ny0 + nmy && pz >= nz0 && pz < nz0 + nmz;
        c[idx] = (inside && !nxt) ? m : 0.0;
    }
}

// Section 2.3.4: conservative tri-cubic interpolation of the parent field U (box B gives the
// parent cell of the patch's first child) onto the patch (n per axis), one thread per parent cell.
// Child (cx, cy, cz) takes the cubic Lagrange interpolant through the 4 parent nodes on its side
// along each axis (x innermost, then y, then z).  The 8 children share the 5^3 parents around the
// cell, so the thread walks them once: for each (oz, oy) the 5 values along x give both children's
// x-sums, which are added into the y-sums of the children whose nodes include oy, and those, once
// complete for an oz, into the z-sums: the same operations in the same order for every child.
__global__ void k_interp_cons(double* __restrict__ out, int n0, int n1, int n2, const double* __restrict__ U, Box B) {
    const int m0 = n0 / 2, m1 = n1 / 2, m2 = n2 / 2;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)m0 * m1 * m2) return;
    int X, Y, Z;
    unflat(idx, m1, m2, X, Y, Z);
    // cubic Lagrange weights at +1/4 through nodes -1, 0, 1, 2; the even child mirrors them: child
    // c on an axis uses node offsets o = k - 2 + c (k = 0..3) with weight w[k] (c = 1) or w[3 - k]
    const double w[4] = {-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0};
    auto wt = [&](int c, int k) { return c ? w[k] : w[3 - k]; };
    double tz[2][2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) tz[a][b][c] = 0.0;
    for (int oz = -2; oz <= 2; ++oz) {
        double ty[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (int oy = -2; oy <= 2; ++oy) {
            double u[5];
            for (int ox = -2; ox <= 2; ++ox) u[ox + 2] = U[box_at(B, X + ox, Y + oy, Z + oz)];
            for (int cx = 0; cx < 2; ++cx) {
                double tx = 0.0;
                for (int kx = 0; kx < 4; ++kx) tx = tx + wt(cx, kx) * u[kx + cx];   // ox = kx - 2 + cx
                for (int cy = 0; cy < 2; ++cy) {
                    const int ky = oy + 2 - cy;
                    if (ky >= 0 && ky < 4) ty[cx][cy] = ty[cx][cy] + wt(cy, ky) * tx;
                }
            }
        }
        for (int cz = 0; cz < 2; ++cz) {
            const int kz = oz + 2 - cz;
            if (kz < 0 || kz > 3) continue;
            for (int cx = 0; cx < 2; ++cx)
                for (int cy = 0; cy < 2; ++cy) tz[cx][cy][cz] = tz[cx][cy][cz] + wt(cz, kz) * ty[cx][cy];
        }
    }
    double v[8];
    double mean = 0.0;
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy)
            for (int cz = 0; cz < 2; ++cz) {
                v[(cx * 2 + cy) * 2 + cz] = tz[cx][cy][cz];
                mean = mean + tz[cx][cy][cz];
            }
    const double shift = U[box_at(B, X, Y, Z)] - mean / 8.0;
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy)
            for (int cz = 0; cz < 2; ++cz)
                out[((size_t)(2 * X + cx) * n1 + (2 * Y + cy)) * n2 + (2 * Z + cz)] = v[(cx * 2 + cy) * 2 + cz] + shift;
}

// out[n^3] = D'[patch] + C; out may be C itself
__global__ void k_patch_add(double* out, const double* __restrict__ d, const double* C, int n0, int n1, int n2) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n0 * n1 * n2) return;
    int x, y, z;
    unflat(idx, n1, n2, x, y, z);
    const size_t di = ((size_t)(x + n0 / 2) * (2 * n1) + (y + n1 / 2)) * (2 * n2) + (z + n2 / 2);
    out[idx] = d[di] + C[idx];
}

// the parent cells under D' (n per axis, box B) that the patch does not cover (the central n/2):
// parent += mean of the 8 children of b (D' array)
__global__ void k_restrict_add(double* __restrict__ parent, Box B, const double* __restrict__ b, int n0, int n1,
                               int n2) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n0 * n1 * n2) return;
    int x, y, z;
    unflat(idx, n1, n2, x, y, z);
    double s = 0.0;
    const int d1 = 2 * n1, d2 = 2 * n2;
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 2; ++e) s = s + b[((size_t)(2 * x + a) * d1 + (2 * y + c)) * d2 + (2 * z + e)];
    const bool cov = x >= n0 / 4 && x < n0 / 4 + n0 / 2 && y >= n1 / 4 && y < n1 / 4 + n1 / 2 && z >= n2 / 4 &&
                     z < n2 / 4 + n2 / 2;
    const size_t pi = box_at(B, x, y, z);
    parent[pi] = parent[pi] + (cov ? 0.0 : s / 8.0);
}



}  // namespace

static bool all_even(const int* P) { return P[0] % 2 == 0 && P[1] % 2 == 0 && P[2] % 2 == 0; }
static size_t octant(const int* P) { return (size_t)(P[0] / 2 + 1) * (P[1] / 2 + 1) * (P[2] / 2 + 1); }

hipError_t launch_kernel_direct(double* T, const int* P, double h, const double* table, double dr, int subgrid,
                                hipStream_t st) {
    if (all_even(P)) {
        k_kernel_direct_oct<<<grid_for(octant(P)), kBlock, 0, st>>>(T, P[0], P[1], P[2], h, table, dr, subgrid);
    } else {
        const size_t n = (size_t)P[0] * P[1] * P[2];
        k_kernel_direct<<<grid_for(n), kBlock, 0, st>>>(T, P[0], P[1], P[2], h, table, dr, subgrid);
    }
    return hipGetLastError();
}

hipError_t launch_kernel_restrict(double* Tc, const int* P, double h, const double* Tf, const int* Pf,
                                  const double* table, double dr, hipStream_t st) {
    if (all_even(P)) {
        k_kernel_restrict_oct<<<grid_for(octant(P)), kBlock, 0, st>>>(Tc, P[0], P[1], P[2], h, Tf, Pf[0], Pf[1],
                                                                     Pf[2], table, dr);
    } else {
        const size_t n = (size_t)P[0] * P[1] * P[2];
        k_kernel_restrict<<<grid_for(n), kBlock, 0, st>>>(Tc, P[0], P[1], P[2], h, Tf, Pf[0], Pf[1], Pf[2], table,
                                                          dr);
    }
    return hipGetLastError();
}

hipError_t launch_divide(double* out, const double* in, size_t n, double d, hipStream_t st) {
    k_divide<<<grid_for(n), kBlock, 0, st>>>(out, in, n, d);
    return hipGetLastError();
}

static Box mkbox(const DensBox& b) {
    Box B;
    for (int a = 0; a < 3; ++a) {
        B.pd[a] = b.pd[a];
        B.po[a] = b.po[a];
        B.lo[a] = b.lo[a];
    }
    B.wrap = b.wrap;
    return B;
}

hipError_t launch_gather(double* dst, const int* n, const double* src, const DensBox& b, hipStream_t st) {
    const size_t c = (size_t)n[0] * n[1] * n[2];
    k_gather<<<grid_for(c), kBlock, 0, st>>>(dst, n[0], n[1], n[2], src, mkbox(b));
    return hipGetLastError();
}

hipError_t launch_restrict_mean(double* parent, const DensBox& b, const int* m, const double* child, const int* cd,
                                const int* co, hipStream_t st) {
    const size_t c = (size_t)m[0] * m[1] * m[2];
    k_restrict_mean<<<grid_for(c), kBlock, 0, st>>>(parent, mkbox(b), m[0], m[1], m[2], child, cd[0], cd[1], cd[2],
                                                    co[0], co[1], co[2]);
    return hipGetLastError();
}

hipError_t launch_zero_box(double* out, const double* in, const int* n, const int* lo, const int* m, hipStream_t st) {
    const size_t c = (size_t)n[0] * n[1] * n[2];
    k_zero_box<<<grid_for(c), kBlock, 0, st>>>(out, in, n[0], n[1], n[2], lo[0], lo[1], lo[2], m[0], m[1], m[2]);
    return hipGetLastError();
}

hipError_t launch_conv_prep(double* a, double* b, double* c, const double* mu, const int* n, const double* par,
                            const DensBox& pb, const int* next_lo, const int* next_m, hipStream_t st) {
    const size_t cnt = (size_t)8 * n[0] * n[1] * n[2];
    const int zero[3] = {0, 0, 0};
    const int* nl = next_lo ? next_lo : zero;
    const int* nm = next_m ? next_m : zero;
    k_conv_prep<<<grid_for(cnt), kBlock, 0, st>>>(a, b, c, mu, n[0], n[1], n[2], par, mkbox(pb), nl[0], nl[1], nl[2],
                                                  nm[0], nm[1], nm[2]);
    return hipGetLastError();
}

hipError_t launch_interp_cons(double* out, const int* n, const double* U, const DensBox& b, hipStream_t st) {
    const size_t c = (size_t)(n[0] / 2) * (n[1] / 2) * (n[2] / 2);
    k_interp_cons<<<grid_for(c), kBlock, 0, st>>>(out, n[0], n[1], n[2], U, mkbox(b));
    return hipGetLastError();
}

hipError_t launch_patch_add(double* out, const double* d, const double* C, const int* n, hipStream_t st) {
    const size_t c = (size_t)n[0] * n[1] * n[2];
    k_patch_add<<<grid_for(c), kBlock, 0, st>>>(out, d, C, n[0], n[1], n[2]);
    return hipGetLastError();
}

hipError_t launch_restrict_add(double* parent, const DensBox& b, const double* bnd, const int* n, hipStream_t st) {
    const size_t c = (size_t)n[0] * n[1] * n[2];
    k_restrict_add<<<grid_for(c), kBlock, 0, st>>>(parent, mkbox(b), bnd, n[0], n[1], n[2]);
    return hipGetLastError();
}

}  // namespace mgic
