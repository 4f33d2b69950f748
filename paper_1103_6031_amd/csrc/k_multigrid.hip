// Multigrid kernels for gfx950: red-black Gauss-Seidel smoothing, residual + restriction,
// FAS coarse right-hand side, prolongation + correction, exact coarsest solve, coarse-fine
// ghost zones with flux matching, composite residual norms and deterministic reductions.
//
// Operators (Hahn & Abel 2011, Section 3.2, Table 1 order 2, summed over the three axes):
//   smoother      u <- (((x- + x+) + (y- + y+)) + (z- + z+) - h^2 f) / 6 on one colour
//   residual      r = f - (neighbour_sum - 6 u) / h^2
//   restriction   mean of the 8 children          prolongation   injection into the 8 children
// Section 3.3: restriction / prolongation only on the region a level shares with the next finer
// one; patches take their boundary values from ghost zones (see k_ghost_fill).
//
// Layout: every level is a row-major [x][y][z] array (z contiguous).  A patch's ghost layer is
// 6 face arrays back to back (mgic::ghost_face_offset).  Compiled with -ffp-contract=off so the
// arithmetic order written here is the order executed.

#include "mg_internal.h"

namespace mgic {

// ----------------------------------------------------------------------------------------------
// neighbour access
// ----------------------------------------------------------------------------------------------

template <class T, bool GH>
__device__ __forceinline__ T neighbour_sum(const T* __restrict__ u, const T* __restrict__ g, Dims d,
                                           int x, int y, int z, size_t i) {
    const size_t sx = (size_t)d.y * d.z;
    const size_t sy = (size_t)d.z;
    T xm, xp, ym, yp, zm, zp;
    if constexpr (GH) {
        xm = x > 0 ? u[i - sx] : g[ghost_face_offset(d, 0) + (size_t)y * d.z + z];
        xp = x < d.x - 1 ? u[i + sx] : g[ghost_face_offset(d, 1) + (size_t)y * d.z + z];
        ym = y > 0 ? u[i - sy] : g[ghost_face_offset(d, 2) + (size_t)x * d.z + z];
        yp = y < d.y - 1 ? u[i + sy] : g[ghost_face_offset(d, 3) + (size_t)x * d.z + z];
        zm = z > 0 ? u[i - 1] : g[ghost_face_offset(d, 4) + (size_t)x * d.y + y];
        zp = z < d.z - 1 ? u[i + 1] : g[ghost_face_offset(d, 5) + (size_t)x * d.y + y];
    } else {
        xm = u[x > 0 ? i - sx : i + (size_t)(d.x - 1) * sx];
        xp = u[x < d.x - 1 ? i + sx : i - (size_t)(d.x - 1) * sx];
        ym = u[y > 0 ? i - sy : i + (size_t)(d.y - 1) * sy];
        yp = u[y < d.y - 1 ? i + sy : i - (size_t)(d.y - 1) * sy];
        zm = u[z > 0 ? i - 1 : i + (size_t)(d.z - 1)];
        zp = u[z < d.z - 1 ? i + 1 : i - (size_t)(d.z - 1)];
    }
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ size_t pidx(const ParentMap& pm, int X, int Y, int Z) {
    // parent index of covered cell (X,Y,Z) relative to the covered box (wraps on periodic parents)
    int a = pm.off[0] + X, b = pm.off[1] + Y, c = pm.off[2] + Z;
    if (pm.periodic) { a = wrap(a, pm.pd.x); b = wrap(b, pm.pd.y); c = wrap(c, pm.pd.z); }
    return ((size_t)a * pm.pd.y + b) * pm.pd.z + c;
}

// ----------------------------------------------------------------------------------------------
// deterministic block reduction (wave64 shuffle, then the 4 waves in order)
// ----------------------------------------------------------------------------------------------

__device__ double block_sum(double v) {
    __shared__ double s_w[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += s_w[k];
    return r;  // valid on thread 0
}

// ----------------------------------------------------------------------------------------------
// elementwise helpers
// ----------------------------------------------------------------------------------------------

template <class T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class A, class B>
__global__ void k_convert(const A* __restrict__ a, B* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = (B)a[i];
}

__global__ void k_add_f32(double* __restrict__ u, const float* __restrict__ e, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        u[i] = u[i] + (double)e[i];
}

template <class T>
__global__ void k_sub_mean(T* __restrict__ a, size_t n, const double* __restrict__ sum, double inv_count) {
    const T m = (T)(sum[0] * inv_count);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = a[i] - m;
}

// ----------------------------------------------------------------------------------------------
// red-black Gauss-Seidel half-sweep: one thread per cell of the colour
// ----------------------------------------------------------------------------------------------

template <class T, bool GH>
__global__ void k_rbgs_half(T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g, Dims d,
                            T h2, int colour) {
    const int nzh = d.z >> 1;
    const size_t total = (size_t)d.x * d.y * nzh;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int zh = (int)(t % nzh);
    const size_t r = t / nzh;
    const int y = (int)(r % d.y);
    const int x = (int)(r / d.y);
    const int z = 2 * zh + ((x + y + colour) & 1);
    const size_t i = ((size_t)x * d.y + y) * d.z + z;
    const T s = neighbour_sum<T, GH>(u, g, d, x, y, z, i);
    u[i] = (s - h2 * f[i]) / T(6);
}

// ----------------------------------------------------------------------------------------------
// residual + restriction (steps 3-5), one thread per covered coarse cell
// ----------------------------------------------------------------------------------------------

template <class T, bool GH>
__global__ void k_resid_restrict(const T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g,
                                 Dims d, T h2, T* __restrict__ pu, T* __restrict__ pf, T* __restrict__ uold,
                                 ParentMap pm) {
    const Dims c{d.x >> 1, d.y >> 1, d.z >> 1};
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= c.cells()) return;
    const int Z = (int)(t % c.z);
    const int Y = (int)((t / c.z) % c.y);
    const int X = (int)(t / ((size_t)c.z * c.y));
    T su = T(0), sr = T(0);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) {
                const int x = 2 * X + a, y = 2 * Y + b, z = 2 * Z + e;
                const size_t i = ((size_t)x * d.y + y) * d.z + z;
                const T ui = u[i];
                const T s = neighbour_sum<T, GH>(u, g, d, x, y, z, i);
                const T lap = (s - T(6) * ui) / h2;
                sr = sr + (f[i] - lap);
                su = su + ui;
            }
    const T uc = su * T(0.125);
    const size_t P = pidx(pm, X, Y, Z);
    pu[P] = uc;
    pf[P] = sr * T(0.125);
    uold[t] = uc;
}

// step 6: parent f[cov] += L u over the parent's stencil
template <class T>
__global__ void k_fas_rhs(const T* __restrict__ pu, T* __restrict__ pf, ParentMap pm, Dims cov, T H2) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= cov.cells()) return;
    const int Z = (int)(t % cov.z);
    const int Y = (int)((t / cov.z) % cov.y);
    const int X = (int)(t / ((size_t)cov.z * cov.y));
    const int a = pm.off[0] + X, b = pm.off[1] + Y, c = pm.off[2] + Z;
    const Dims d = pm.pd;
    const size_t i = ((size_t)wrap(a, d.x) * d.y + wrap(b, d.y)) * d.z + wrap(c, d.z);
    const T s = neighbour_sum<T, false>(pu, nullptr, d, wrap(a, d.x), wrap(b, d.y), wrap(c, d.z), i);
    pf[i] = pf[i] + (s - T(6) * pu[i]) / H2;
}

// step 8: u += inject(parent u[cov] - uold)
template <class T>
__global__ void k_prolong(T* __restrict__ u, Dims d, const T* __restrict__ pu, const T* __restrict__ uold,
                          ParentMap pm) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= d.cells()) return;
    const int z = (int)(t % d.z);
    const int y = (int)((t / d.z) % d.y);
    const int x = (int)(t / ((size_t)d.z * d.y));
    const int X = x >> 1, Y = y >> 1, Z = z >> 1;
    const size_t o = ((size_t)X * (d.y >> 1) + Y) * (d.z >> 1) + Z;
    u[t] = u[t] + (pu[pidx(pm, X, Y, Z)] - uold[o]);
}

// step 1: exact zero-mean solve on an odd periodic M^3 grid by its discrete Green's function,
// G(d) = M^-3 sum_{m != 0} cos(2 pi m.d / M) / lambda(m), lambda the 7-point symbol (Table 1).
template <class T>
__global__ void k_coarsest(T* __restrict__ u, const T* __restrict__ f, int M, double h) {
    __shared__ double G[343];
    __shared__ double F[343];
    const int n3 = M * M * M;
    if (M == 1) {
        if (threadIdx.x == 0) u[0] = T(0);
        return;
    }
    const double inv_h2 = 1.0 / (h * h);
    for (int t = threadIdx.x; t < n3; t += blockDim.x) {
        const int dz = t % M, dy = (t / M) % M, dx = t / (M * M);
        double acc = 0.0;
        for (int m = 1; m < n3; ++m) {
            const int mz = m % M, my = (m / M) % M, mx = m / (M * M);
            const double lam = -2.0 * inv_h2 *
                               ((1.0 - cospi(2.0 * mx / M)) + (1.0 - cospi(2.0 * my / M)) + (1.0 - cospi(2.0 * mz / M)));
            const int ph = (mx * dx + my * dy + mz * dz) % M;
            acc += cospi(2.0 * ph / M) / lam;
        }
        G[t] = acc / n3;
        F[t] = (double)f[t];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n3; t += blockDim.x) {
        const int z = t % M, y = (t / M) % M, x = t / (M * M);
        double acc = 0.0;
        for (int s = 0; s < n3; ++s) {
            const int sz = s % M, sy = (s / M) % M, sx = s / (M * M);
            const int dx = (x - sx + M) % M, dy = (y - sy + M) % M, dz = (z - sz + M) % M;
            acc += G[(dx * M + dy) * M + dz] * F[s];
        }
        u[t] = (T)acc;
    }
}

// ----------------------------------------------------------------------------------------------
// coarse-fine ghost zones with flux matching (Section 3.3, Table 2 order-1 flux), one thread per
// 2x2 group of fine face cells sharing a parent C.  For the low-x face and fine cell (0, j, k):
//   a  = quadratic interpolation in the outside parent layer at the child's transverse position
//   g0 = 8/15 a + 2/3 u0 - 1/5 u1            (quadratic normal to the face)
//   g  = g0 + (mean u0 - mean g0) - 1/2 (mean8(children of C) - U[O])
// so the mean fine flux (u0 - g)/h through the coarse face equals the coarse flux (C - O)/(2h),
// with C taken as the live mean of its children.  Other faces mirror this.
// ----------------------------------------------------------------------------------------------

__device__ __forceinline__ void w2(double t, double w[3]) {
    w[0] = 0.5 * t * (t - 1.0);
    w[1] = 1.0 - t * t;
    w[2] = 0.5 * t * (t + 1.0);
}

template <class T>
__global__ void k_ghost_fill(const T* __restrict__ pu, const T* __restrict__ u, T* __restrict__ g, Dims d,
                             ParentMap pm, int flux_match) {
    const int n[3] = {d.x, d.y, d.z};
    const size_t gx = (size_t)(d.y / 2) * (d.z / 2), gy = (size_t)(d.x / 2) * (d.z / 2),
                 gz = (size_t)(d.x / 2) * (d.y / 2);
    size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    int face;
    if (t < 2 * gx) face = (int)(t / gx), t %= gx;
    else if ((t -= 2 * gx) < 2 * gy) face = 2 + (int)(t / gy), t %= gy;
    else if ((t -= 2 * gy) < 2 * gz) face = 4 + (int)(t / gz), t %= gz;
    else return;
    const int a = face >> 1, side = face & 1;
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    const int nc2 = n[c] / 2;
    const int J = (int)(t / nc2), K = (int)(t % nc2);
    // fine interior layers and the outside coarse layer along the face normal
    const int i0 = side ? n[a] - 1 : 0, i1 = side ? n[a] - 2 : 1;
    const int on = side ? pm.off[a] + n[a] / 2 : pm.off[a] - 1;
    const int pdim[3] = {pm.pd.x, pm.pd.y, pm.pd.z};
    // 3x3 outside coarse layer around O
    double L[3][3];
    for (int db = 0; db < 3; ++db)
        for (int dc = 0; dc < 3; ++dc) {
            int q[3];
            q[a] = on;
            q[b] = pm.off[b] + J + db - 1;
            q[c] = pm.off[c] + K + dc - 1;
            if (pm.periodic) for (int k = 0; k < 3; ++k) q[k] = wrap(q[k], pdim[k]);
            L[db][dc] = (double)pu[((size_t)q[0] * pdim[1] + q[1]) * pdim[2] + q[2]];
        }
    double u0[2][2], u1[2][2], g0[2][2];
    for (int jb = 0; jb < 2; ++jb)
        for (int kc = 0; kc < 2; ++kc) {
            int p0[3], p1[3];
            p0[a] = i0; p1[a] = i1;
            p0[b] = p1[b] = 2 * J + jb;
            p0[c] = p1[c] = 2 * K + kc;
            u0[jb][kc] = (double)u[((size_t)p0[0] * d.y + p0[1]) * d.z + p0[2]];
            u1[jb][kc] = (double)u[((size_t)p1[0] * d.y + p1[1]) * d.z + p1[2]];
            double wb[3], wc[3];
            w2(jb ? 0.25 : -0.25, wb);
            w2(kc ? 0.25 : -0.25, wc);
            // parallel to the face: first along b (for each of the 3 c-columns), then along c
            double Ab[3];
            for (int dc = 0; dc < 3; ++dc) Ab[dc] = (wb[0] * L[0][dc] + wb[1] * L[1][dc]) + wb[2] * L[2][dc];
            const double aq = (wc[0] * Ab[0] + wc[1] * Ab[1]) + wc[2] * Ab[2];
            g0[jb][kc] = ((8.0 / 15.0) * aq + (2.0 / 3.0) * u0[jb][kc]) - 0.2 * u1[jb][kc];
        }
    double shift = 0.0;
    if (flux_match) {
        const double m_u0 = ((u0[0][0] + u0[0][1]) + (u0[1][0] + u0[1][1])) * 0.25;
        const double m_u1 = ((u1[0][0] + u1[0][1]) + (u1[1][0] + u1[1][1])) * 0.25;
        const double m_g0 = ((g0[0][0] + g0[0][1]) + (g0[1][0] + g0[1][1])) * 0.25;
        const double uC = 0.5 * (m_u0 + m_u1);
        shift = (m_u0 - m_g0) - 0.5 * (uC - L[1][1]);
    }
    const size_t fo = ghost_face_offset(d, face);
    const int nbf = n[c];  // face arrays are [n_b][n_c]
    for (int jb = 0; jb < 2; ++jb)
        for (int kc = 0; kc < 2; ++kc)
            g[fo + (size_t)(2 * J + jb) * nbf + (2 * K + kc)] = (T)(g0[jb][kc] + shift);
}

// parent[cov] = mean8(fine), bottom-up composite restriction
template <class T>
__global__ void k_restrict_cov(const T* __restrict__ v, Dims d, T* __restrict__ pv, ParentMap pm) {
    const Dims c{d.x >> 1, d.y >> 1, d.z >> 1};
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= c.cells()) return;
    const int Z = (int)(t % c.z);
    const int Y = (int)((t / c.z) % c.y);
    const int X = (int)(t / ((size_t)c.z * c.y));
    T s = T(0);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) s = s + v[((size_t)(2 * X + a) * d.y + (2 * Y + b)) * d.z + (2 * Z + e)];
    pv[pidx(pm, X, Y, Z)] = s * T(0.125);
}

// ----------------------------------------------------------------------------------------------
// residual of a level with optional output, partial sums of r^2 outside the covered box
// ----------------------------------------------------------------------------------------------

__device__ __forceinline__ bool in_box(const CovBox& cb, int x, int y, int z) {
    return (unsigned)(x - cb.lo[0]) < (unsigned)cb.n[0] && (unsigned)(y - cb.lo[1]) < (unsigned)cb.n[1] &&
           (unsigned)(z - cb.lo[2]) < (unsigned)cb.n[2];
}

template <class T, class R, bool GH>
__global__ void k_residual(const T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g, Dims d,
                           T h2, CovBox cb, R* __restrict__ rout, double* __restrict__ partials) {
    double acc = 0.0;
    const size_t n = d.cells();
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % d.z);
        const int y = (int)((i / d.z) % d.y);
        const int x = (int)(i / ((size_t)d.z * d.y));
        const T s = neighbour_sum<T, GH>(u, g, d, x, y, z, i);
        const T r = f[i] - (s - T(6) * u[i]) / h2;
        const bool cov = in_box(cb, x, y, z);
        if (!cov) acc += (double)r * (double)r;
        if (rout) rout[i] = cov ? R(0) : (R)r;
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

__global__ void k_sum(const double* __restrict__ a, Dims d, CovBox cb, int square, double* __restrict__ partials) {
    double acc = 0.0;
    const size_t n = d.cells();
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % d.z);
        const int y = (int)((i / d.z) % d.y);
        const int x = (int)(i / ((size_t)d.z * d.y));
        if (in_box(cb, x, y, z)) continue;
        const double v = a[i];
        acc += square ? v * v : v;
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

__global__ void k_finalize(const double* __restrict__ partials, SegList segs, double* __restrict__ out) {
    double total = 0.0;
    for (int s = 0; s < segs.n; ++s) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < segs.cnt[s]; i += blockDim.x) acc += partials[segs.off[s] + i];
        const double bs = block_sum(acc);
        if (threadIdx.x == 0) total += segs.w[s] * bs;
    }
    if (threadIdx.x == 0) out[0] = total;
}

// ----------------------------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------------------------

template <class T>
void launch_fill(T* p, size_t n, T v, hipStream_t st) {
    k_fill<T><<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(p, n, v);
}
template <class A, class B>
void launch_convert(const A* a, B* b, size_t n, hipStream_t st) {
    k_convert<A, B><<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(a, b, n);
}
void launch_add_f32_to_f64(double* u, const float* e, size_t n, hipStream_t st) {
    k_add_f32<<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(u, e, n);
}
template <class T>
void launch_sub_mean(T* a, size_t n, const double* sum, double inv_count, hipStream_t st) {
    k_sub_mean<T><<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(a, n, sum, inv_count);
}

template <class T>
void launch_rbgs_half(T* u, const T* f, const T* ghosts, Dims d, double h, int colour, hipStream_t st) {
    const size_t n = (size_t)d.x * d.y * (d.z / 2);
    const T h2 = (T)(h * h);
    if (ghosts)
        k_rbgs_half<T, true><<<grid_for(n), kBlock, 0, st>>>(u, f, ghosts, d, h2, colour);
    else
        k_rbgs_half<T, false><<<grid_for(n), kBlock, 0, st>>>(u, f, nullptr, d, h2, colour);
}

template <class T>
void launch_resid_restrict(const T* u, const T* f, const T* ghosts, Dims d, double h, T* pu, T* pf, T* uold,
                           ParentMap pm, hipStream_t st) {
    const size_t n = (size_t)(d.x / 2) * (d.y / 2) * (d.z / 2);
    const T h2 = (T)(h * h);
    if (ghosts)
        k_resid_restrict<T, true><<<grid_for(n), kBlock, 0, st>>>(u, f, ghosts, d, h2, pu, pf, uold, pm);
    else
        k_resid_restrict<T, false><<<grid_for(n), kBlock, 0, st>>>(u, f, nullptr, d, h2, pu, pf, uold, pm);
}

template <class T>
void launch_fas_rhs(const T* pu, T* pf, ParentMap pm, Dims cov, double H, hipStream_t st) {
    k_fas_rhs<T><<<grid_for(cov.cells()), kBlock, 0, st>>>(pu, pf, pm, cov, (T)(H * H));
}

template <class T>
void launch_prolong(T* u, Dims d, const T* pu, const T* uold, ParentMap pm, hipStream_t st) {
    k_prolong<T><<<grid_for(d.cells()), kBlock, 0, st>>>(u, d, pu, uold, pm);
}

template <class T>
void launch_coarsest(T* u, const T* f, int M, double h, hipStream_t st) {
    k_coarsest<T><<<1, kBlock, 0, st>>>(u, f, M, h);
}

template <class T>
void launch_ghost_fill(const T* pu, const T* u, T* ghosts, Dims d, ParentMap pm, int flux_match, hipStream_t st) {
    const size_t n = 2 * ((size_t)(d.y / 2) * (d.z / 2) + (size_t)(d.x / 2) * (d.z / 2) + (size_t)(d.x / 2) * (d.y / 2));
    k_ghost_fill<T><<<grid_for(n), kBlock, 0, st>>>(pu, u, ghosts, d, pm, flux_match);
}

template <class T>
void launch_restrict_cov(const T* fine, Dims d, T* parent, ParentMap pm, hipStream_t st) {
    const size_t n = (size_t)(d.x / 2) * (d.y / 2) * (d.z / 2);
    k_restrict_cov<T><<<grid_for(n), kBlock, 0, st>>>(fine, d, parent, pm);
}

template <class T, class R>
void launch_residual(const T* u, const T* f, const T* ghosts, Dims d, double h, CovBox cov, R* rout,
                     double* partials, int* nparts, hipStream_t st) {
    const int g = grid_for(d.cells(), kBlock, kMaxPartials);
    const T h2 = (T)(h * h);
    if (ghosts)
        k_residual<T, R, true><<<g, kBlock, 0, st>>>(u, f, ghosts, d, h2, cov, rout, partials);
    else
        k_residual<T, R, false><<<g, kBlock, 0, st>>>(u, f, nullptr, d, h2, cov, rout, partials);
    *nparts = g;
}

void launch_sum(const double* a, Dims d, CovBox cov, int square, double* partials, int* nparts, hipStream_t st) {
    const int g = grid_for(d.cells(), kBlock, kMaxPartials);
    k_sum<<<g, kBlock, 0, st>>>(a, d, cov, square, partials);
    *nparts = g;
}

void launch_finalize(const double* partials, SegList segs, double* out, hipStream_t st) {
    k_finalize<<<1, kBlock, 0, st>>>(partials, segs, out);
}

// explicit instantiations
template void launch_fill<double>(double*, size_t, double, hipStream_t);
template void launch_fill<float>(float*, size_t, float, hipStream_t);
template void launch_convert<double, float>(const double*, float*, size_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, size_t, hipStream_t);
template void launch_convert<double, double>(const double*, double*, size_t, hipStream_t);
template void launch_sub_mean<double>(double*, size_t, const double*, double, hipStream_t);
#define MGIC_INST(T)                                                                                          \
    template void launch_rbgs_half<T>(T*, const T*, const T*, Dims, double, int, hipStream_t);                \
    template void launch_resid_restrict<T>(const T*, const T*, const T*, Dims, double, T*, T*, T*, ParentMap, \
                                           hipStream_t);                                                      \
    template void launch_fas_rhs<T>(const T*, T*, ParentMap, Dims, double, hipStream_t);                      \
    template void launch_prolong<T>(T*, Dims, const T*, const T*, ParentMap, hipStream_t);                    \
    template void launch_coarsest<T>(T*, const T*, int, double, hipStream_t);                                 \
    template void launch_ghost_fill<T>(const T*, const T*, T*, Dims, ParentMap, int, hipStream_t);            \
    template void launch_restrict_cov<T>(const T*, Dims, T*, ParentMap, hipStream_t);
MGIC_INST(double)
MGIC_INST(float)
#undef MGIC_INST
template void launch_residual<double, double>(const double*, const double*, const double*, Dims, double, CovBox,
                                              double*, double*, int*, hipStream_t);
template void launch_residual<double, float>(const double*, const double*, const double*, Dims, double, CovBox,
                                             float*, double*, int*, hipStream_t);

}  // namespace mgic
