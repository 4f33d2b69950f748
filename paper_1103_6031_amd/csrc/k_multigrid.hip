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
// Storage (mgic::Lay): every level is [x][y][z] by rows of z.  Periodic levels with an even z
// extent use the colour-split row layout: the red cells ((x+y+z) even) of a row first, in
// increasing z, then its black cells.  A red/black half-sweep then reads and writes unit-stride
// runs only, and the 8 children of a coarse cell sit at the same position Z of both halves of 4
// fine rows.  Patches (natural rows) keep a separate ghost layer of 6 faces.
// Compiled with -ffp-contract=off so the arithmetic order written here is the order executed.

#include <hip/hip_ext.h>

#include <algorithm>

#include "mg_internal.h"
#include "p2_bodies.h"

namespace mgic {

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }


// ((x- + x+) + (y- + y+)) + (z- + z+) on a periodic level in any layout
template <class T>
__device__ __forceinline__ T nsum_periodic(const T* __restrict__ u, Dims d, int sp, int x, int y, int z) {
    const T xm = u[lidx(d, sp, wrap(x - 1, d.x), y, z)], xp = u[lidx(d, sp, wrap(x + 1, d.x), y, z)];
    const T ym = u[lidx(d, sp, x, wrap(y - 1, d.y), z)], yp = u[lidx(d, sp, x, wrap(y + 1, d.y), z)];
    const T zm = u[lidx(d, sp, x, y, wrap(z - 1, d.z))], zp = u[lidx(d, sp, x, y, wrap(z + 1, d.z))];
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// the same on a patch (in its layout, natural or colour-split) whose outside neighbours come from
// the ghost faces
template <class T>
__device__ __forceinline__ T nsum_ghost(const T* __restrict__ u, const T* __restrict__ g, const Lay& L, int x, int y,
                                        int z) {
    const Dims d = L.d;
    const T xm = x > 0 ? u[lidx(L, x - 1, y, z)] : g[ghost_face_offset(d, 0) + (size_t)y * d.z + z];
    const T xp = x < d.x - 1 ? u[lidx(L, x + 1, y, z)] : g[ghost_face_offset(d, 1) + (size_t)y * d.z + z];
    const T ym = y > 0 ? u[lidx(L, x, y - 1, z)] : g[ghost_face_offset(d, 2) + (size_t)x * d.z + z];
    const T yp = y < d.y - 1 ? u[lidx(L, x, y + 1, z)] : g[ghost_face_offset(d, 3) + (size_t)x * d.z + z];
    const T zm = z > 0 ? u[lidx(L, x, y, z - 1)] : g[ghost_face_offset(d, 4) + (size_t)x * d.y + y];
    const T zp = z < d.z - 1 ? u[lidx(L, x, y, z + 1)] : g[ghost_face_offset(d, 5) + (size_t)x * d.y + y];
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

template <class T, bool GH>
__device__ __forceinline__ T nsum(const T* __restrict__ u, const T* __restrict__ g, const Lay& L, int x, int y,
                                  int z) {
    if constexpr (GH) return nsum_ghost<T>(u, g, L, x, y, z);
    else return nsum_periodic<T>(u, L.d, L.split, x, y, z);
}

// index of covered cell (X,Y,Z) (relative to the covered box) in the parent array
__device__ __forceinline__ size_t pidx(const ParentMap& pm, int X, int Y, int Z) {
    int a = pm.off[0] + X, b = pm.off[1] + Y, c = pm.off[2] + Z;
    if (pm.periodic) {
        a = wrap(a, pm.pl.d.x);
        b = wrap(b, pm.pl.d.y);
        c = wrap(c, pm.pl.d.z);
    }
    return lidx(pm.pl.d, pm.pl.split, a, b, c);
}


// Reduction kernels stride over the whole array, kRedV independent cells per thread per pass;
// blk / nblk are the block's index and the block count of its array (the grid of a plain launch,
// the instance's share of a batched one).  (Measured on MI355X: giving each block one contiguous
// chunk instead was no faster.)
__device__ __forceinline__ unsigned red_lo(unsigned blk) { return blk * blockDim.x * kRedV; }
__device__ __forceinline__ unsigned red_stride(unsigned nblk) { return nblk * blockDim.x * kRedV; }
// The reductions that read neighbours (residuals, the outer step) give each block one contiguous
// range of whole passes (blockDim.x * kRedV cells each) instead of striding over the grid: the
// rows above and below a block's rows are its own, and the neighbour planes are read by blocks a
// plane's range away, dispatched at about the same time (on the same XCD when that distance is a
// multiple of 8), so they are still in L2.  Fixed by (blk, nblk, n), so the sums stay deterministic.
struct RedRange {
    unsigned lo, hi, stride;
};
__device__ __forceinline__ RedRange red_range(unsigned blk, unsigned nblk, unsigned n) {
    const unsigned per = blockDim.x * kRedV;
    const unsigned passes = ((n + per - 1) / per + nblk - 1) / nblk;
    const unsigned lo = blk * passes * per;
    return RedRange{lo, lo < n ? min(n, lo + passes * per) : n, per};
}

// ----------------------------------------------------------------------------------------------
// deterministic block reduction (wave64 shuffle, then the waves in order)
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

// dst (layout ld) = src (layout ls), converting the element type
template <class A, class B>
__global__ void k_relayout(const A* __restrict__ src, Lay ls, B* __restrict__ dst, Lay ld) {
    const size_t n = ld.d.cells();
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        ldecode(ld, i, x, y, z);
        dst[i] = (B)src[lidx(ls, x, y, z)];
    }
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
// per-cell bodies shared by the grid-wide kernels and the single-workgroup tail kernel (so both
// produce the same bits)
// ----------------------------------------------------------------------------------------------

// split-layout half-sweep of the cell t of `colour` (t = (row, j) over rows of nz/2 cells).
// Indices are 32-bit: every level fits in 2^31 cells.
// The general colour-split half-sweep runs in plane-chunk order, 8 blocks per x plane, when a
// plane's cells of one colour fill at least 8 passes of a block of `block` threads and fewer
// than 16 blocks of block V cells.  Measured against flat order: 96^3 solves FP64 2.01 -> 1.93
// ms, mixed 1.69 -> 1.67 ms; the 64 batched instances of 32^3-128^3 13.02 -> 12.85-12.95 ms.
// With 32 chunks per plane a 192^3 mixed solve went 3.34 -> 3.48 ms, so larger planes keep flat
// order.
__host__ __device__ inline bool split_chunked(const Lay& L, unsigned block, unsigned V) {
    const size_t hp = (size_t)L.d.y * (size_t)(L.d.z >> 1);
    return !L.pow2 && hp >= 8u * (size_t)block && hp < 16u * (size_t)block * V;
}

// blocks of a general colour-split half-sweep: d.x * 8 in plane-chunk order, else n / (block V)
unsigned rbgs_split_blocks(const Lay& L, int block, int V) {
    if (split_chunked(L, (unsigned)block, (unsigned)V)) return (unsigned)L.d.x * 8u;
    const size_t n = (size_t)L.d.x * L.d.y * (L.d.z / 2);
    return (unsigned)((n + (size_t)block * V - 1) / ((size_t)block * V));
}

template <class T>
__device__ __forceinline__ void cell_rbgs_split(T* __restrict__ u, const T* __restrict__ f, const Lay& L, T h2,
                                                int colour, unsigned t) {
    const Dims d = L.d;
    const unsigned nzh = (unsigned)d.z >> 1;
    unsigned j, r0, rxm, rxp, rym, ryp, jm, jp;
    int q;                                       // z parity of this colour in the row
    if (L.pow2) {   // power-of-two level: the same indices by shifts and masks
        const unsigned lzh = (unsigned)L.lgz - 1, mx = (unsigned)d.x - 1, my = (unsigned)d.y - 1;
        const unsigned row = t >> lzh;
        j = t & (nzh - 1);
        const unsigned x = row >> L.lgy, y = row & my;
        q = (int)((x + y + (unsigned)colour) & 1u);
        r0 = row << L.lgz;
        rxm = ((((x - 1) & mx) << L.lgy) | y) << L.lgz;
        rxp = ((((x + 1) & mx) << L.lgy) | y) << L.lgz;
        rym = ((x << L.lgy) | ((y - 1) & my)) << L.lgz;
        ryp = ((x << L.lgy) | ((y + 1) & my)) << L.lgz;
        jm = (j - 1 + (unsigned)q) & (nzh - 1);
        jp = (j + (unsigned)q) & (nzh - 1);
    } else {
        const unsigned row = L.dzh.div(t);
        j = t - row * nzh;
        const unsigned xq = L.dy.div(row);
        const int y = (int)(row - xq * (unsigned)d.y);
        const int x = (int)xq;
        q = (x + y + colour) & 1;
        const unsigned rs = (unsigned)d.z;
        rxm = ((unsigned)wrap(x - 1, d.x) * d.y + y) * rs;
        rxp = ((unsigned)wrap(x + 1, d.x) * d.y + y) * rs;
        rym = ((unsigned)x * d.y + wrap(y - 1, d.y)) * rs;
        ryp = ((unsigned)x * d.y + wrap(y + 1, d.y)) * rs;
        r0 = row * rs;
        // the cell is z = 2j + q; its z-neighbours are the other colour's entries (z-1)/2, (z+1)/2
        jm = (unsigned)wrap((int)j - 1 + q, (int)nzh);
        jp = (unsigned)wrap((int)j + q, (int)nzh);
    }
    const unsigned own = colour ? nzh : 0u, oth = colour ? 0u : nzh;
    const T xm = u[rxm + oth + j], xp = u[rxp + oth + j];
    const T ym = u[rym + oth + j], yp = u[ryp + oth + j];
    const T zm = u[r0 + oth + jm], zp = u[r0 + oth + jp];
    const T s = ((xm + xp) + (ym + yp)) + (zm + zp);
    u[r0 + own + j] = (s - h2 * f[r0 + own + j]) / T(6);
}

// residual + restriction of the covered coarse cell t (steps 3-5)
template <class T, bool GH>
__device__ __forceinline__ void cell_resid_restrict(const T* __restrict__ u, const T* __restrict__ f,
                                                    const T* __restrict__ g, const Lay& L, T h2,
                                                    T* __restrict__ pu, T* __restrict__ pf,
                                                    T* __restrict__ uold, const ParentMap& pm, const Lay& C,
                                                    unsigned t) {
    int X, Y, Z;
    ldecode(C, t, X, Y, Z);   // C: the covered box (natural order)
    T su = T(0), sr = T(0);
    if constexpr (GH) {
        // the ghost-face neighbour sums are branchy: unrolling all 8 children spills registers;
        // the children are taken in the same (a, b, e) order as below
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const int x = 2 * X + (k >> 2), y = 2 * Y + ((k >> 1) & 1), z = 2 * Z + (k & 1);
            const size_t i = lidx(L, x, y, z);
            const T ui = u[i];
            const T s = nsum<T, GH>(u, g, L, x, y, z);
            const T lap = (s - T(6) * ui) / h2;
            sr = sr + (f[i] - lap);
            su = su + ui;
        }
    } else {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e) {
                    const int x = 2 * X + a, y = 2 * Y + b, z = 2 * Z + e;
                    const size_t i = lidx(L, x, y, z);
                    const T ui = u[i];
                    const T s = nsum<T, GH>(u, g, L, x, y, z);
                    const T lap = (s - T(6) * ui) / h2;
                    sr = sr + (f[i] - lap);
                    su = su + ui;
                }
    }
    const T uc = su * T(0.125);
    const size_t P = pidx(pm, X, Y, Z);
    pu[P] = uc;
    pf[P] = sr * T(0.125);
    uold[t] = uc;
}

// step 6 for covered cell t: parent f += L u over the parent's own (periodic-wrapped) stencil
template <class T>
__device__ __forceinline__ void cell_fas(const T* __restrict__ pu, T* __restrict__ pf, const ParentMap& pm,
                                         const Lay& C, T H2, unsigned t) {
    int X, Y, Z;
    ldecode(C, t, X, Y, Z);   // C: the covered box (natural order)
    const int a = wrap(pm.off[0] + X, pm.pl.d.x), b = wrap(pm.off[1] + Y, pm.pl.d.y), c = wrap(pm.off[2] + Z, pm.pl.d.z);
    const size_t i = lidx(pm.pl.d, pm.pl.split, a, b, c);
    const T s = nsum_periodic<T>(pu, pm.pl.d, pm.pl.split, a, b, c);
    pf[i] = pf[i] + (s - T(6) * pu[i]) / H2;
}

// step 8 for the fine cell at storage position t: u += parent u[cov] - uold
template <class T>
__device__ __forceinline__ void cell_prolong(T* __restrict__ u, const Lay& L, const T* __restrict__ pu,
                                             const T* __restrict__ uold, const ParentMap& pm, unsigned t) {
    int x, y, z;
    ldecode(L, t, x, y, z);
    const int X = x >> 1, Y = y >> 1, Z = z >> 1;
    const size_t o = ((size_t)X * (L.d.y >> 1) + Y) * (L.d.z >> 1) + Z;
    u[t] = u[t] + (pu[pidx(pm, X, Y, Z)] - uold[o]);
}

// step 1 on an odd periodic M^3 grid (M <= 7) by one workgroup: the discrete Green's function
// G(d) = M^-3 sum_{m != 0} cos(2 pi m.d / M) / lambda(m), lambda the 7-point symbol (Table 1).
// G and F are workgroup arrays of at least M^3 doubles.
template <class T>
__device__ void block_coarsest(T* __restrict__ u, const T* __restrict__ f, int M, double h, double* G, double* F) {
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
// grid-wide kernels
// ----------------------------------------------------------------------------------------------

// periodic level in the colour-split layout.  In plane-chunk order (split_chunked) the plane's
// cells of the colour are cut into 8 contiguous, equal chunks and block blk takes chunk blk mod 8
// of plane blk / 8.  Consecutive blocks go to the 8 XCDs in turn, so the blocks holding the same
// chunk of neighbouring planes are 8 apart and share an XCD, whose L2 then already holds the
// x-neighbour rows a block reads.  In flat order (9 blocks per plane at
// 96^3, for instance) they sit on different XCDs and every x-neighbour row is fetched again:
// counters read 2.1x the algorithmic bytes for a 96^3 FP32 half-sweep.  Otherwise V consecutive
// cells of a half-row per thread in flat order.  Every cell's update is the same either way.
template <class T, int V>
__device__ __forceinline__ void body_rbgs_split(T* __restrict__ u, const T* __restrict__ f, const Lay& L, T h2,
                                                int colour, unsigned blk) {
    if (split_chunked(L, blockDim.x, V)) {
        const unsigned hp = (unsigned)L.d.y * ((unsigned)L.d.z >> 1);
        const unsigned chunk = (hp + 7u) >> 3;
        const unsigned lo = (blk & 7u) * chunk, hi = min(lo + chunk, hp);
        const unsigned base = (blk >> 3) * hp;
        for (unsigned t = lo + threadIdx.x; t < hi; t += blockDim.x) cell_rbgs_split<T>(u, f, L, h2, colour, base + t);
        return;
    }
    const unsigned total = (unsigned)L.d.x * L.d.y * ((unsigned)L.d.z >> 1);
    const unsigned base = blk * blockDim.x * V + threadIdx.x;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const unsigned t = base + v * blockDim.x;   // each of the V passes is unit-stride over the wave
        if (t < total) cell_rbgs_split<T>(u, f, L, h2, colour, t);
    }
}

template <class T, int V>
__global__ void k_rbgs_split(T* __restrict__ u, const T* __restrict__ f, Lay L, T h2, int colour) {
    body_rbgs_split<T, V>(u, f, L, h2, colour, (unsigned)xcd_block());
}

// patch in the colour-split layout with ghost faces: one thread per cell of the colour, the cell
// (x, y, j) of a row is z = 2j + ((x + y + colour) & 1); neighbours inside the patch are the other
// colour's entries of the neighbour rows, outside ones come from the ghost faces
template <class T>
__global__ void k_rbgs_ghost(T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g, Lay L, T h2,
                             int colour) {
    const Dims d = L.d;
    const unsigned nzh = (unsigned)d.z >> 1;
    const unsigned total = (unsigned)d.x * d.y * nzh;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const unsigned row = L.dzh.div(t);
    const unsigned j = t - row * nzh;
    const unsigned xq = L.dy.div(row);
    const int y = (int)(row - xq * (unsigned)d.y);
    const int x = (int)xq;
    const int q = (x + y + colour) & 1;
    const int z = 2 * (int)j + q;
    const unsigned own = colour ? nzh : 0u, oth = colour ? 0u : nzh;
    const unsigned rs = (unsigned)d.z;
    const unsigned r0 = row * rs;
    const T xm = x > 0 ? u[r0 - (unsigned)d.y * rs + oth + j] : g[ghost_face_offset(d, 0) + (size_t)y * d.z + z];
    const T xp = x < d.x - 1 ? u[r0 + (unsigned)d.y * rs + oth + j] : g[ghost_face_offset(d, 1) + (size_t)y * d.z + z];
    const T ym = y > 0 ? u[r0 - rs + oth + j] : g[ghost_face_offset(d, 2) + (size_t)x * d.z + z];
    const T yp = y < d.y - 1 ? u[r0 + rs + oth + j] : g[ghost_face_offset(d, 3) + (size_t)x * d.z + z];
    // z-neighbours z -+ 1 are the other colour's entries (z - 1) / 2 and (z + 1) / 2
    const T zm = z > 0 ? u[r0 + oth + (unsigned)((z - 1) >> 1)] : g[ghost_face_offset(d, 4) + (size_t)x * d.y + y];
    const T zp = z < d.z - 1 ? u[r0 + oth + (unsigned)((z + 1) >> 1)] : g[ghost_face_offset(d, 5) + (size_t)x * d.y + y];
    const T s = ((xm + xp) + (ym + yp)) + (zm + zp);
    u[r0 + own + j] = (s - h2 * f[r0 + own + j]) / T(6);
}

// k_rbgs_ghost on runs of W cells of the colour in one half-row (W = 4 in FP32, 2 in FP64), as
// run_rbgs_vec on periodic levels: the x- and y-neighbour runs, f and the other colour's entries
// of the own row are 16-byte loads.  In rows on a face the neighbours outside the patch come from
// that face's ghosts (the run's cells sit at every second z), and the two ends of a row from the
// z faces.  Half-rows hold a multiple of W cells and the arrays are 16-byte aligned.  Each cell
// has the operations of k_rbgs_ghost, so the bits are the same.
template <class T>
__global__ void k_rbgs_ghost_vec(T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g, Lay L, T h2,
                                 int colour) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    const Dims d = L.d;
    const unsigned nzh = (unsigned)d.z >> 1;
    const unsigned ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= (unsigned)d.x * d.y * (nzh / W)) return;
    const unsigned t = ch * W;                 // first cell of the run in the colour's order
    const unsigned row = L.dzh.div(t);
    const unsigned j0 = t - row * nzh;
    const unsigned xq = L.dy.div(row);
    const int y = (int)(row - xq * (unsigned)d.y), x = (int)xq;
    const unsigned q = (unsigned)(x + y + colour) & 1u;
    const unsigned own = colour ? nzh : 0u, oth = colour ? 0u : nzh;
    const unsigned rs = (unsigned)d.z, r0 = row * rs;
    const unsigned zb = 2 * j0 + q;            // z of the run's cell k is zb + 2k
    auto face_run = [&](int face, size_t line) {
        const T* p = g + ghost_face_offset(d, face) + line + zb;
        T v[W];
#pragma unroll
        for (int k = 0; k < W; ++k) v[k] = p[2 * k];
        if constexpr (W == 4) return V{v[0], v[1], v[2], v[3]};
        else return V{v[0], v[1]};
    };
    const V C = *(const V*)(u + r0 + oth + j0);
    const V F = *(const V*)(f + r0 + own + j0);
    // the z-neighbour outside the run: entry j0 - 1 (q = 0) or j0 + W (q = 1) of the other colour,
    // or the z face's ghost at the ends of the row (one load from either address)
    const bool zin = q ? j0 + W < nzh : j0 > 0;
    const T* ep = zin ? u + (r0 + oth + (q ? j0 + W : j0 - 1))
                      : g + ghost_face_offset(d, 4 + (int)q) + (size_t)x * d.y + y;
    const T edge = *ep;
    auto sweep = [&](const V& XM, const V& XP, const V& YM, const V& YP) {
        T out[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const T zm = q ? lane<T>(C, k) : (k == 0 ? edge : lane<T>(C, k - 1));
            const T zp = q ? (k == W - 1 ? edge : lane<T>(C, k + 1)) : lane<T>(C, k);
            const T s = ((lane<T>(XM, k) + lane<T>(XP, k)) + (lane<T>(YM, k) + lane<T>(YP, k))) + (zm + zp);
            out[k] = (s - h2 * lane<T>(F, k)) / T(6);
        }
        V o;
        if constexpr (W == 4) o = V{out[0], out[1], out[2], out[3]};
        else o = V{out[0], out[1]};
        *(V*)(u + r0 + own + j0) = o;
    };
    if (x > 0 && x < d.x - 1 && y > 0 && y < d.y - 1) {   // rows off the x and y faces: no branch
        const V XM = *(const V*)(u + r0 - (unsigned)d.y * rs + oth + j0);
        const V XP = *(const V*)(u + r0 + (unsigned)d.y * rs + oth + j0);
        const V YM = *(const V*)(u + r0 - rs + oth + j0);
        const V YP = *(const V*)(u + r0 + rs + oth + j0);
        sweep(XM, XP, YM, YP);
        return;
    }
    const V XM = x > 0 ? *(const V*)(u + r0 - (unsigned)d.y * rs + oth + j0) : face_run(0, (size_t)y * d.z);
    const V XP = x < d.x - 1 ? *(const V*)(u + r0 + (unsigned)d.y * rs + oth + j0) : face_run(1, (size_t)y * d.z);
    const V YM = y > 0 ? *(const V*)(u + r0 - rs + oth + j0) : face_run(2, (size_t)x * d.z);
    const V YP = y < d.y - 1 ? *(const V*)(u + r0 + rs + oth + j0) : face_run(3, (size_t)x * d.z);
    sweep(XM, XP, YM, YP);
}

template <class T, bool GH>
__global__ void k_resid_restrict(const T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g,
                                 Lay L, T h2, T* __restrict__ pu, T* __restrict__ pf, T* __restrict__ uold,
                                 ParentMap pm, Lay C) {
    const unsigned n = (unsigned)C.d.cells();
    const unsigned t = (unsigned)xcd_block() * blockDim.x + threadIdx.x;
    if (t < n) cell_resid_restrict<T, GH>(u, f, g, L, h2, pu, pf, uold, pm, C, t);
}

// Steps 3-5 of a colour-split patch for covered cell t (natural order of the covered box), with
// every load of the 8 children issued before any sum, as cell_resid_restrict_p2 on periodic
// levels: the four central rows (x0 + a, y0 + b) at z0 - 1 .. z0 + 2, f at z0 and z0 + 1, and the
// rows one step outside in x and in y at z0, z0 + 1.  A neighbour outside the patch is read from
// its face's ghosts instead (one load from either address).  The children and their sums are
// taken in the order of cell_resid_restrict, so the bits are the same.
template <class T>
__global__ void k_resid_restrict_gh(const T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g,
                                    Lay L, T h2, T* __restrict__ pu, T* __restrict__ pf, T* __restrict__ uold,
                                    ParentMap pm, Lay C) {
    const unsigned t = (unsigned)xcd_block() * blockDim.x + threadIdx.x;
    if (t >= (unsigned)C.d.cells()) return;
    int X, Y, Z;
    ldecode(C, t, X, Y, Z);
    const Dims d = L.d;
    const int nzh = d.z >> 1;
    const int x0 = 2 * X, y0 = 2 * Y;
    auto rowb = [&](int x, int y) { return ((size_t)x * d.y + y) * d.z; };
    auto half = [&](int x, int y, int zpar) { return (size_t)((x + y + zpar) & 1) * nzh; };
    const size_t f4 = ghost_face_offset(d, 4), f5 = ghost_face_offset(d, 5);
    T cm[2][2], c0[2][2], c1[2][2], c2[2][2], f0[2][2], f1[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int x = x0 + a, y = y0 + b;
            const size_t rb = rowb(x, y), he = half(x, y, 0), ho = half(x, y, 1);
            const size_t gz = (size_t)x * d.y + y;
            cm[a][b] = *(Z > 0 ? u + (rb + ho + Z - 1) : g + (f4 + gz));
            c0[a][b] = u[rb + he + Z];
            c1[a][b] = u[rb + ho + Z];
            c2[a][b] = *(Z + 1 < nzh ? u + (rb + he + Z + 1) : g + (f5 + gz));
            f0[a][b] = f[rb + he + Z];
            f1[a][b] = f[rb + ho + Z];
        }
    T xf[2][2][2], yf[2][2][2];   // [side][b or a][e]
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int z = 2 * Z + e;
                {
                    const int x = sd ? x0 + 2 : x0 - 1, y = y0 + k;
                    const bool in = sd ? x < d.x : x >= 0;
                    xf[sd][k][e] = *(in ? u + (rowb(x, y) + half(x, y, e) + Z)
                                        : g + (ghost_face_offset(d, sd) + (size_t)y * d.z + z));
                }
                {
                    const int x = x0 + k, y = sd ? y0 + 2 : y0 - 1;
                    const bool in = sd ? y < d.y : y >= 0;
                    yf[sd][k][e] = *(in ? u + (rowb(x, y) + half(x, y, e) + Z)
                                        : g + (ghost_face_offset(d, 2 + sd) + (size_t)x * d.z + z));
                }
            }
    auto val = [&](int a, int b, int e) { return e ? c1[a][b] : c0[a][b]; };
    T sr = T(0), su = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const T ui = val(a, b, e);
                const T xm = a ? val(0, b, e) : xf[0][b][e];
                const T xp = a ? xf[1][b][e] : val(1, b, e);
                const T ym = b ? val(a, 0, e) : yf[0][a][e];
                const T yp = b ? yf[1][a][e] : val(a, 1, e);
                const T zm = e ? c0[a][b] : cm[a][b];
                const T zp = e ? c2[a][b] : c1[a][b];
                const T s = ((xm + xp) + (ym + yp)) + (zm + zp);
                const T lap = (s - T(6) * ui) / h2;
                sr = sr + ((e ? f1[a][b] : f0[a][b]) - lap);
                su = su + ui;
            }
    const T uc = su * T(0.125);
    const size_t P = pidx(pm, X, Y, Z);
    pu[P] = uc;
    pf[P] = sr * T(0.125);
    uold[t] = uc;
}

template <class T>
__global__ void k_fas_rhs(const T* __restrict__ pu, T* __restrict__ pf, ParentMap pm, Lay C, T H2) {
    const unsigned t = (unsigned)xcd_block() * blockDim.x + threadIdx.x;
    if (t < (unsigned)C.d.cells()) cell_fas<T>(pu, pf, pm, C, H2, t);
}

template <class T>
__global__ void k_prolong(T* __restrict__ u, Lay L, const T* __restrict__ pu, const T* __restrict__ uold,
                          ParentMap pm) {
    const unsigned t = (unsigned)xcd_block() * blockDim.x + threadIdx.x;
    if (t < (unsigned)L.d.cells()) cell_prolong<T>(u, L, pu, uold, pm, t);
}

// step 8 on the black cells of a colour-split level only: when a red half-sweep follows, it
// overwrites every red cell without reading it, so correcting the red cells would be dead work
template <class T>
__device__ __forceinline__ void cell_prolong_black(T* __restrict__ u, const Lay& L, const T* __restrict__ pu,
                                                   const T* __restrict__ uold, const ParentMap& pm, unsigned t) {
    const unsigned nzh = (unsigned)L.d.z >> 1;
    const unsigned row = L.dzh.div(t);
    const unsigned j = t - row * nzh;
    const unsigned xq = L.dy.div(row);
    const int y = (int)(row - xq * (unsigned)L.d.y), x = (int)xq;
    const int z = 2 * (int)j + ((x + y + 1) & 1);
    const size_t i = (size_t)row * L.d.z + nzh + j;
    const int X = x >> 1, Y = y >> 1, Z = z >> 1;
    const size_t o = ((size_t)X * (L.d.y >> 1) + Y) * (L.d.z >> 1) + Z;
    u[i] = u[i] + (pu[pidx(pm, X, Y, Z)] - uold[o]);
}

template <class T>
__global__ void k_prolong_black(T* __restrict__ u, Lay L, const T* __restrict__ pu, const T* __restrict__ uold,
                                ParentMap pm) {
    const unsigned t = (unsigned)xcd_block() * blockDim.x + threadIdx.x;
    if (t < (unsigned)(L.d.cells() >> 1)) cell_prolong_black<T>(u, L, pu, uold, pm, t);
}

template <class T>
__global__ void k_coarsest(T* __restrict__ u, const T* __restrict__ f, int M, double h) {
    __shared__ double G[343];
    __shared__ double F[343];
    block_coarsest<T>(u, f, M, h, G, F);
}

// ----------------------------------------------------------------------------------------------
// tail: the whole V-cycle below a small level, run by one workgroup in one launch, with every
// level of it held in LDS.  As separate kernels these levels are launch-bound; here each step is
// a loop of the workgroup's threads over a level's cells with a barrier between steps.  The
// first level's u and f are read from global memory and its u is written back at the end.
// ----------------------------------------------------------------------------------------------

// Copy of a block-uniform value whose 32-bit words are marked wave-uniform, so that the compiler
// keeps it in scalar registers even when it was read from LDS or global memory.
template <class S>
__device__ __forceinline__ S uniform(const S& v) {
    static_assert(sizeof(S) % 4 == 0, "uniform() copies 32-bit words");
    int w[sizeof(S) / 4];
    __builtin_memcpy(w, &v, sizeof(S));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(S) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    S out;
    __builtin_memcpy(&out, w, sizeof(S));
    return out;
}

template <class T>
__device__ void body_tail(const TailPlan<T>& tp) {
    extern __shared__ __align__(16) unsigned char smem[];
    auto U = [&](int k) { return (T*)(smem + uniform(tp.lev[k].lds_u)); };
    auto F = [&](int k) { return (T*)(smem + uniform(tp.lev[k].lds_f)); };
    auto O = [&](int k) { return (T*)(smem + uniform(tp.lev[k].lds_o)); };
    double* G = (double*)(smem + uniform(tp.lds_bytes) - 2 * 343 * sizeof(double));
    double* Gf = G + 343;
    const unsigned nt = blockDim.x;
    {
        const unsigned n0 = (unsigned)uniform(tp.lev[0].lay.d).cells();
        T* U0 = U(0);
        T* F0 = F(0);
        const T* u0g = uniform(tp.lev[0].u);
        const T* f0g = uniform(tp.lev[0].f);
        for (unsigned t = threadIdx.x; t < n0; t += nt) {
            U0[t] = u0g[t];
            F0[t] = f0g[t];
        }
        __syncthreads();
        if (uniform(tp.fas0)) {   // the parent's step 6 on this level: f += L u
            const Lay A = uniform(tp.lev[0].lay);
            const double h0 = uniform(tp.lev[0].h);
            const T H2 = (T)(h0 * h0);
            for (unsigned t = threadIdx.x; t < n0; t += nt) {
                int x, y, z;
                ldecode(A, t, x, y, z);
                const T s = nsum_periodic<T>(U0, A.d, A.split, x, y, z);
                F0[t] = F0[t] + (s - T(6) * U0[t]) / H2;
            }
            __syncthreads();
        }
    }
    // descent: smooth, restrict, FAS right-hand side
    const int nlev = uniform(tp.n), nu1 = uniform(tp.nu1), nu2 = uniform(tp.nu2);
    for (int l = 0; l + 1 < nlev; ++l) {
        const Lay A = uniform(tp.lev[l].lay), Bl = uniform(tp.lev[l + 1].lay);
        const double hl = uniform(tp.lev[l].h);
        const T h2 = (T)(hl * hl);
        const unsigned half = (unsigned)A.d.cells() >> 1;
        for (int s = 0; s < nu1; ++s)
            for (int c = 0; c < 2; ++c) {
                for (unsigned t = threadIdx.x; t < half; t += nt) cell_rbgs_split<T>(U(l), F(l), A, h2, c, t);
                __syncthreads();
            }
        const ParentMap pm(Bl, 0, 0, 0, 1);
        Lay C = Bl;   // the coarse level is the whole covered box, decoded in natural order
        C.split = 0;
        const unsigned nc = (unsigned)A.d.cells() >> 3;
        for (unsigned t = threadIdx.x; t < nc; t += nt)
            cell_resid_restrict<T, false>(U(l), F(l), (const T*)nullptr, A, h2, U(l + 1), F(l + 1), O(l), pm, C, t);
        __syncthreads();
        const double hc = uniform(tp.lev[l + 1].h);
        const T H2 = (T)(hc * hc);
        for (unsigned t = threadIdx.x; t < nc; t += nt) cell_fas<T>(U(l + 1), F(l + 1), pm, C, H2, t);
        __syncthreads();
    }
    {
        const int c = nlev - 1;
        block_coarsest<T>(U(c), F(c), uniform(tp.lev[c].lay.d).x, uniform(tp.lev[c].h), G, Gf);
        __syncthreads();
    }
    // ascent: correct, smooth
    for (int l = nlev - 2; l >= 0; --l) {
        const Lay A = uniform(tp.lev[l].lay), Bl = uniform(tp.lev[l + 1].lay);
        const ParentMap pm(Bl, 0, 0, 0, 1);
        const unsigned n = (unsigned)A.d.cells();
        if (nu2 > 0 && A.split)   // red cells are rewritten unread by the first red half-sweep
            for (unsigned t = threadIdx.x; t < n >> 1; t += nt) cell_prolong_black<T>(U(l), A, U(l + 1), O(l), pm, t);
        else
            for (unsigned t = threadIdx.x; t < n; t += nt) cell_prolong<T>(U(l), A, U(l + 1), O(l), pm, t);
        __syncthreads();
        const double hl = uniform(tp.lev[l].h);
        const T h2 = (T)(hl * hl);
        for (int s = 0; s < nu2; ++s)
            for (int c = 0; c < 2; ++c) {
                for (unsigned t = threadIdx.x; t < n >> 1; t += nt) cell_rbgs_split<T>(U(l), F(l), A, h2, c, t);
                __syncthreads();
            }
    }
    const unsigned n0 = (unsigned)uniform(tp.lev[0].lay.d).cells();
    T* u0out = uniform(tp.lev[0].u);
    for (unsigned t = threadIdx.x; t < n0; t += nt) u0out[t] = U(0)[t];
}

template <class T>
__global__ void __launch_bounds__(kTailThreads) k_tail(TailPlan<T> tp) {
    body_tail<T>(tp);
}

// The same tail when every level but the single-cell coarsest is a colour-split power-of-two cube
// (the coarsenings of a power-of-two base).  Positions and periodic neighbour sums are formed by
// shifts and masks of the edge's log2, and the residual + restriction takes one thread per fine
// cell: the 8 children of a coarse cell sit in 8 neighbouring lanes and are summed by lane
// shuffles in the same (a, b, e) order.  The operations on every value are those of body_tail,
// so the bits are the same; only the index arithmetic and the work split differ.
__device__ __forceinline__ unsigned p2pos(int lg, unsigned x, unsigned y, unsigned z) {
    if (lg == 0) return 0u;   // the single-cell coarsest level
    return ((((x << lg) | y) << lg) + (((x + y + z) & 1u) << (lg - 1))) + (z >> 1);
}

template <class T>
__device__ __forceinline__ T p2nsum(const T* u, int lg, unsigned x, unsigned y, unsigned z) {
    const unsigned m = (1u << lg) - 1;
    const T xm = u[p2pos(lg, (x - 1) & m, y, z)], xp = u[p2pos(lg, (x + 1) & m, y, z)];
    const T ym = u[p2pos(lg, x, (y - 1) & m, z)], yp = u[p2pos(lg, x, (y + 1) & m, z)];
    const T zm = u[p2pos(lg, x, y, (z - 1) & m)], zp = u[p2pos(lg, x, y, (z + 1) & m)];
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

template <class T>
__device__ void body_tail_p2(const TailPlan<T>& tp) {
    extern __shared__ __align__(16) unsigned char smem[];
    auto U = [&](int k) { return (T*)(smem + uniform(tp.lev[k].lds_u)); };
    auto F = [&](int k) { return (T*)(smem + uniform(tp.lev[k].lds_f)); };
    auto O = [&](int k) { return (T*)(smem + uniform(tp.lev[k].lds_o)); };
    const unsigned nt = blockDim.x, tid = threadIdx.x;
    const int nlev = uniform(tp.n), nu1 = uniform(tp.nu1), nu2 = uniform(tp.nu2);
    const int lg0 = uniform(tp.lev[0].lay.lgx);
    {
        const unsigned n0 = 1u << (3 * lg0);
        T* U0 = U(0);
        T* F0 = F(0);
        const T* u0g = uniform(tp.lev[0].u);
        const T* f0g = uniform(tp.lev[0].f);
        for (unsigned t = tid; t < n0; t += nt) {
            U0[t] = u0g[t];
            F0[t] = f0g[t];
        }
        __syncthreads();
        if (uniform(tp.fas0)) {   // the parent's step 6 on this level: f += L u
            const Lay A = uniform(tp.lev[0].lay);
            const double h0 = uniform(tp.lev[0].h);
            const T H2 = (T)(h0 * h0);
            for (unsigned t = tid; t < n0; t += nt) {
                int x, y, z;
                ldecode(A, t, x, y, z);
                const T s = p2nsum<T>(U0, lg0, (unsigned)x, (unsigned)y, (unsigned)z);
                F0[t] = F0[t] + (s - T(6) * U0[t]) / H2;
            }
            __syncthreads();
        }
    }
    for (int l = 0; l + 1 < nlev; ++l) {
        const Lay A = uniform(tp.lev[l].lay);
        const int lg = lg0 - l, lc = lg - 1;
        const double hl = uniform(tp.lev[l].h);
        const T h2 = (T)(hl * hl);
        const unsigned n = 1u << (3 * lg), half = n >> 1, mc = (1u << lc) - 1;
        T* u = U(l);
        T* f = F(l);
        T* pu = U(l + 1);
        T* pf = F(l + 1);
        T* uo = O(l);
        for (int s = 0; s < nu1; ++s)
            for (int c = 0; c < 2; ++c) {
                for (unsigned t = tid; t < half; t += nt) cell_rbgs_split<T>(u, f, A, h2, c, t);
                __syncthreads();
            }
        for (unsigned base = 0; base < n; base += nt) {   // every lane of a wave takes part in the shuffles
            const unsigned t = base + tid, ch = t & 7, cc = t >> 3;
            const bool act = t < n;
            const unsigned X = cc >> (2 * lc), Y = (cc >> lc) & mc, Z = cc & mc;
            const unsigned x = 2 * X + (ch >> 2), y = 2 * Y + ((ch >> 1) & 1), z = 2 * Z + (ch & 1);
            T r = T(0), ui = T(0);
            if (act) {
                const unsigned i = p2pos(lg, x, y, z);
                ui = u[i];
                const T sn = p2nsum<T>(u, lg, x, y, z);
                const T lap = (sn - T(6) * ui) / h2;
                r = f[i] - lap;
            }
            const int lane0 = (int)(tid & 63) & ~7;
            T sr = T(0), su = T(0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                sr = sr + __shfl(r, lane0 + q, 64);
                su = su + __shfl(ui, lane0 + q, 64);
            }
            if (act && ch == 0) {
                const T uc = su * T(0.125);
                const unsigned P = p2pos(lc, X, Y, Z);
                pu[P] = uc;
                pf[P] = sr * T(0.125);
                uo[cc] = uc;
            }
        }
        __syncthreads();
        const double hc = uniform(tp.lev[l + 1].h);
        const T H2 = (T)(hc * hc);
        for (unsigned t = tid; t < (n >> 3); t += nt) {
            const unsigned X = t >> (2 * lc), Y = (t >> lc) & mc, Z = t & mc;
            const unsigned i = p2pos(lc, X, Y, Z);
            const T sn = p2nsum<T>(pu, lc, X, Y, Z);
            pf[i] = pf[i] + (sn - T(6) * pu[i]) / H2;
        }
        __syncthreads();
    }
    if (tid == 0) U(nlev - 1)[0] = T(0);   // step 1 on the single-cell coarsest level
    __syncthreads();
    for (int l = nlev - 2; l >= 0; --l) {
        const Lay A = uniform(tp.lev[l].lay);
        const int lg = lg0 - l, lc = lg - 1;
        const unsigned n = 1u << (3 * lg), m = (1u << lg) - 1, nzh = 1u << (lg - 1);
        T* u = U(l);
        const T* pu = U(l + 1);
        const T* uo = O(l);
        if (nu2 > 0) {   // red cells are rewritten unread by the first red half-sweep
            for (unsigned t = tid; t < (n >> 1); t += nt) {
                const unsigned row = t >> (lg - 1), j = t & (nzh - 1);
                const unsigned x = row >> lg, y = row & m, z = 2 * j + ((x + y + 1) & 1);
                const unsigned i = (row << lg) + nzh + j;
                const unsigned X = x >> 1, Y = y >> 1, Z = z >> 1;
                u[i] = u[i] + (pu[p2pos(lc, X, Y, Z)] - uo[(((X << lc) | Y) << lc) | Z]);
            }
        } else {
            for (unsigned t = tid; t < n; t += nt) {
                int x, y, z;
                ldecode(A, t, x, y, z);
                const unsigned X = (unsigned)x >> 1, Y = (unsigned)y >> 1, Z = (unsigned)z >> 1;
                u[t] = u[t] + (pu[p2pos(lc, X, Y, Z)] - uo[(((X << lc) | Y) << lc) | Z]);
            }
        }
        __syncthreads();
        const double hl = uniform(tp.lev[l].h);
        const T h2 = (T)(hl * hl);
        for (int s = 0; s < nu2; ++s)
            for (int c = 0; c < 2; ++c) {
                for (unsigned t = tid; t < (n >> 1); t += nt) cell_rbgs_split<T>(u, F(l), A, h2, c, t);
                __syncthreads();
            }
    }
    const unsigned n0 = 1u << (3 * lg0);
    T* u0out = uniform(tp.lev[0].u);
    for (unsigned t = tid; t < n0; t += nt) u0out[t] = U(0)[t];
}

template <class T>
__global__ void __launch_bounds__(kTailThreads) k_tail_p2(TailPlan<T> tp) {
    body_tail_p2<T>(tp);
}

// ----------------------------------------------------------------------------------------------
// coarse-fine ghost zones with flux matching (Section 3.3, Table 2 order-1 flux), computed per 2x2
// group of fine face cells sharing a parent C.  For the low-x face and fine cell (0, j, k):
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

// The ghost value of lane q = 2 jb + kc (jb, kc in {0, 1}) of group (J, K) on face `face` of a
// patch: the group is the 2 x 2 fine ghost cells in front of parent cell (J, K) of the face (J
// along axis b, K along axis c; a is the normal).  Each lane forms its own g0; the group means
// are gathered by lane shuffles in the order ((q0 + q1) + (q2 + q3)), the order of the sums
// written out over the group, so the bits do not depend on how the group is split over lanes.
// The four lanes of a group must be consecutive lanes of one wave starting at a multiple of 4,
// and every lane of the wave must take part (lanes with no group of their own repeat a valid one).
// The parent's part of the value - the interpolation aq in the outside parent layer and the
// parent cell O in front of the group - does not change while the patch alone is smoothed:
// MODE 1 also returns it in pa = {aq, O}, MODE 2 takes it from pa instead of the parent.
template <class T, int MODE>
__device__ __forceinline__ double ghost_lane(const T* __restrict__ pu, const T* __restrict__ u, const Lay& LF,
                                             const ParentMap& pm, int face, int J, int K, int q, int flux_match,
                                             double2& pa) {
    const Dims d = LF.d;
    const int n[3] = {d.x, d.y, d.z};
    const int a = face >> 1, side = face & 1;
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    const int jb = q >> 1, kc = q & 1;
    // fine interior layers and the outside coarse layer along the face normal
    const int i0 = side ? n[a] - 1 : 0, i1 = side ? n[a] - 2 : 1;
    int p0[3], p1[3];
    p0[a] = i0;
    p1[a] = i1;
    p0[b] = p1[b] = 2 * J + jb;
    p0[c] = p1[c] = 2 * K + kc;
    const double u0 = (double)u[lidx(LF, p0[0], p0[1], p0[2])];
    const double u1 = (double)u[lidx(LF, p1[0], p1[1], p1[2])];
    double aq, O;
    if constexpr (MODE == 2) {
        aq = pa.x;
        O = pa.y;
    } else {
        const int on = side ? pm.off[a] + n[a] / 2 : pm.off[a] - 1;
        const int pdim[3] = {pm.pl.d.x, pm.pl.d.y, pm.pl.d.z};
        // 3x3 outside coarse layer around O
        double L[3][3];
        for (int db = 0; db < 3; ++db)
            for (int dc = 0; dc < 3; ++dc) {
                int qq[3];
                qq[a] = on;
                qq[b] = pm.off[b] + J + db - 1;
                qq[c] = pm.off[c] + K + dc - 1;
                if (pm.periodic)
                    for (int k = 0; k < 3; ++k) qq[k] = wrap(qq[k], pdim[k]);
                L[db][dc] = (double)pu[lidx(pm.pl.d, pm.pl.split, qq[0], qq[1], qq[2])];
            }
        double wb[3], wc[3];
        w2(jb ? 0.25 : -0.25, wb);
        w2(kc ? 0.25 : -0.25, wc);
        // parallel to the face: first along b (for each of the 3 c-columns), then along c
        double Ab[3];
        for (int dc = 0; dc < 3; ++dc) Ab[dc] = (wb[0] * L[0][dc] + wb[1] * L[1][dc]) + wb[2] * L[2][dc];
        aq = (wc[0] * Ab[0] + wc[1] * Ab[1]) + wc[2] * Ab[2];
        O = L[1][1];
        if constexpr (MODE == 1) pa = make_double2(aq, O);
    }
    const double g0 = ((8.0 / 15.0) * aq + (2.0 / 3.0) * u0) - 0.2 * u1;
    double shift = 0.0;
    if (flux_match) {
        const int base = (int)(threadIdx.x & 63) & ~3;
        auto mean4 = [&](double v) {
            const double v0 = __shfl(v, base, 64), v1 = __shfl(v, base + 1, 64);
            const double v2 = __shfl(v, base + 2, 64), v3 = __shfl(v, base + 3, 64);
            return ((v0 + v1) + (v2 + v3)) * 0.25;
        };
        const double m_u0 = mean4(u0), m_u1 = mean4(u1), m_g0 = mean4(g0);
        const double uC = 0.5 * (m_u0 + m_u1);
        shift = (m_u0 - m_g0) - 0.5 * (uC - O);
    }
    return g0 + shift;
}

// One lane per ghost cell, four lanes per group (ghost_lane), one launch row per face.  Four
// short chains instead of one long one, and four times the waves, for a launch that is
// latency-bound.  MODE 1 stores each cell's parent part in pa (indexed as the ghosts), MODE 2
// reads it back: the fills after the first of a smoothing pass skip the parent layer.
template <class T, int MODE>
__global__ void k_ghost_fill(const T* __restrict__ pu, const T* __restrict__ u, T* __restrict__ g,
                             double2* __restrict__ pa, Lay LF, ParentMap pm, int flux_match) {
    const Dims d = LF.d;
    const int n[3] = {d.x, d.y, d.z};
    const int face = (int)blockIdx.y;
    const int a = face >> 1;
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    const unsigned nc2 = (unsigned)n[c] / 2;
    const unsigned lane = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned t = lane >> 2, q = lane & 3;
    // lanes past the face compute on a valid group (the last one) and store nothing
    const unsigned ngroups = ((unsigned)n[b] / 2) * nc2;
    const bool live = t < ngroups;
    const unsigned tg = live ? t : ngroups - 1;
    const int J = (int)(tg / nc2), K = (int)(tg - (unsigned)J * nc2);
    const size_t gi = ghost_face_offset(d, face) + (size_t)(2 * J + (int)(q >> 1)) * n[c] + (2 * K + (int)(q & 1));
    double2 part = make_double2(0.0, 0.0);
    if constexpr (MODE == 2) part = pa[gi];
    const double v = ghost_lane<T, MODE>(pu, u, LF, pm, face, J, K, (int)q, flux_match, part);
    if (!live) return;
    g[gi] = (T)v;   // face arrays are [n_b][n_c]
    if constexpr (MODE == 1) pa[gi] = part;
}

// parent[cov] = mean8(fine), bottom-up composite restriction
template <class T>
__global__ void k_restrict_cov(const T* __restrict__ v, Lay L, T* __restrict__ pv, ParentMap pm) {
    const Dims c{L.d.x >> 1, L.d.y >> 1, L.d.z >> 1};
    const size_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= c.cells()) return;
    const int Z = (int)(t % c.z);
    const int Y = (int)((t / c.z) % c.y);
    const int X = (int)(t / ((size_t)c.z * c.y));
    T s = T(0);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) s = s + v[lidx(L, 2 * X + a, 2 * Y + b, 2 * Z + e)];
    pv[pidx(pm, X, Y, Z)] = s * T(0.125);
}

// Storage position t of a colour-split periodic level (either colour): its coordinates and the
// storage rows of its six neighbours, wrapped.  Power-of-two levels use shifts and masks.
struct SplitNb {
    unsigned j, col, oth, r0, rxm, rxp, rym, ryp, jm, jp;
    int x, y, q;
};
__device__ __forceinline__ SplitNb split_nb(const Lay& L, unsigned t) {
    const Dims d = L.d;
    const unsigned nz = (unsigned)d.z, nzh = nz >> 1;
    SplitNb c;
    unsigned row, p;
    if (L.pow2) {
        row = t >> L.lgz;
        p = t & (nz - 1);
        c.x = (int)(row >> L.lgy);
        c.y = (int)(row & ((unsigned)d.y - 1));
    } else {
        row = L.dz.div(t);
        p = t - row * nz;
        const unsigned xq = L.dy.div(row);
        c.y = (int)(row - xq * (unsigned)d.y);
        c.x = (int)xq;
    }
    c.col = p >= nzh;
    c.j = p - c.col * nzh;
    c.q = (c.x + c.y + (int)c.col) & 1;
    c.oth = c.col ? 0u : nzh;
    if (L.pow2) {
        const unsigned mx = (unsigned)d.x - 1, my = (unsigned)d.y - 1, x = (unsigned)c.x, y = (unsigned)c.y;
        c.r0 = row << L.lgz;
        c.rxm = ((((x - 1) & mx) << L.lgy) | y) << L.lgz;
        c.rxp = ((((x + 1) & mx) << L.lgy) | y) << L.lgz;
        c.rym = ((x << L.lgy) | ((y - 1) & my)) << L.lgz;
        c.ryp = ((x << L.lgy) | ((y + 1) & my)) << L.lgz;
        c.jm = (c.j - 1 + (unsigned)c.q) & (nzh - 1);
        c.jp = (c.j + (unsigned)c.q) & (nzh - 1);
    } else {
        c.r0 = row * nz;
        c.rxm = ((unsigned)wrap(c.x - 1, d.x) * d.y + c.y) * nz;
        c.rxp = ((unsigned)wrap(c.x + 1, d.x) * d.y + c.y) * nz;
        c.rym = ((unsigned)c.x * d.y + wrap(c.y - 1, d.y)) * nz;
        c.ryp = ((unsigned)c.x * d.y + wrap(c.y + 1, d.y)) * nz;
        c.jm = (unsigned)wrap((int)c.j - 1 + c.q, (int)nzh);
        c.jp = (unsigned)wrap((int)c.j + c.q, (int)nzh);
    }
    return c;
}

// ----------------------------------------------------------------------------------------------
// residual of a level with optional output, partial sums of r^2 outside the covered box
// ----------------------------------------------------------------------------------------------

__device__ __forceinline__ bool in_box(const CovBox& cb, int x, int y, int z) {
    return (unsigned)(x - cb.lo[0]) < (unsigned)cb.n[0] && (unsigned)(y - cb.lo[1]) < (unsigned)cb.n[1] &&
           (unsigned)(z - cb.lo[2]) < (unsigned)cb.n[2];
}

template <class T, class R, bool GH>
__device__ __forceinline__ double body_residual(const T* __restrict__ u, const T* __restrict__ f,
                                                const T* __restrict__ g, const Lay& L, T h2, const CovBox& cb,
                                                R* __restrict__ rout, const Lay& LR, unsigned blk, unsigned nblk) {
    double acc = 0.0;
    const size_t n = L.d.cells();
    const RedRange rr = red_range(blk, nblk, (unsigned)n);
    const unsigned lo = rr.lo, hi = rr.hi, stride = rr.stride;
    for (unsigned b0 = lo + threadIdx.x; b0 < hi; b0 += stride)
#pragma unroll
    for (int v = 0; v < kRedV; ++v) {
        const unsigned i = b0 + v * blockDim.x;
        if (i >= hi) break;
        int x, y, z;
        ldecode(L, i, x, y, z);
        const T s = nsum<T, GH>(u, g, L, x, y, z);
        const T r = f[i] - (s - T(6) * u[i]) / h2;
        const bool cov = in_box(cb, x, y, z);
        if (!cov) acc += (double)r * (double)r;
        if (rout) rout[lidx(LR, x, y, z)] = cov ? R(0) : (R)r;
    }
    return acc;
}

template <class T, class R, bool GH>
__global__ void k_residual(const T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ g, Lay L,
                           T h2, CovBox cb, R* __restrict__ rout, Lay LR, double* __restrict__ partials) {
    const double bs = block_sum(body_residual<T, R, GH>(u, f, g, L, h2, cb, rout, LR, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// the same on a colour-split periodic level, r written in the same layout; neighbour rows are
// addressed directly (identical arithmetic, so identical bits)
template <class T, class R>
__device__ __forceinline__ double body_residual_split(const T* __restrict__ u, const T* __restrict__ f,
                                                      const Lay& L, T h2, const CovBox& cb, R* __restrict__ rout,
                                                      unsigned blk, unsigned nblk) {
    const Dims d = L.d;
    const unsigned n = (unsigned)d.cells(), nz = (unsigned)d.z, nzh = nz >> 1;
    double acc = 0.0;
    const RedRange rr = red_range(blk, nblk, (unsigned)n);
    const unsigned lo = rr.lo, hi = rr.hi, stride = rr.stride;
    // FP64, no covered box, no output and even half-rows: pairs of cells with 16-byte runs (the
    // loads of the outer step's pairs), each cell with the same operations as below
    if constexpr (sizeof(T) == 8) {
        if (!rout && (cb.n[0] <= 0 || cb.n[1] <= 0 || cb.n[2] <= 0) && (nzh & 1u) == 0) {
            for (unsigned p0 = lo; p0 < hi; p0 += stride)
#pragma unroll
            for (int v = 0; v < kRedV / 2; ++v) {
                const unsigned t = p0 + 2 * (threadIdx.x + v * blockDim.x);
                if (t >= hi) break;
                const SplitNb c = split_nb(L, t);
                const unsigned j = c.j, oth = c.oth, r0 = c.r0, q = (unsigned)c.q;
                const double2 fv = *(const double2*)(f + t);
                const unsigned ix[6] = {t, c.rxm + oth + j, c.rxp + oth + j, c.rym + oth + j, c.ryp + oth + j,
                                        r0 + oth + j};
                const unsigned jn = q ? j + 2 : j + nzh - 1;
                const unsigned ie = r0 + oth + (jn >= nzh ? jn - nzh : jn);
                double2 w[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) w[k] = *(const double2*)(u + ix[k]);
                const double edge = u[ie];
                __builtin_amdgcn_sched_barrier(0);
                const double zm0 = q ? w[5].x : edge, zp0 = q ? w[5].y : w[5].x;
                const double zm1 = q ? w[5].y : w[5].x, zp1 = q ? edge : w[5].y;
                const double s0 = ((w[1].x + w[2].x) + (w[3].x + w[4].x)) + (zm0 + zp0);
                const double s1 = ((w[1].y + w[2].y) + (w[3].y + w[4].y)) + (zm1 + zp1);
                const double ra = fv.x - (s0 - 6.0 * w[0].x) / (double)h2;
                const double rb = fv.y - (s1 - 6.0 * w[0].y) / (double)h2;
                acc += ra * ra;
                acc += rb * rb;
            }
            return acc;
        }
    }
    for (unsigned b0 = lo + threadIdx.x; b0 < hi; b0 += stride)
#pragma unroll
    for (int v = 0; v < kRedV; ++v) {
        const unsigned t = b0 + v * blockDim.x;
        if (t >= hi) break;
        const SplitNb c = split_nb(L, t);
        const unsigned j = c.j, col = c.col, oth = c.oth, r0 = c.r0, rxm = c.rxm, rxp = c.rxp, rym = c.rym,
                       ryp = c.ryp, jm = c.jm, jp = c.jp;
        const int x = c.x, y = c.y, q = c.q;
        const T s = ((u[rxm + oth + j] + u[rxp + oth + j]) + (u[rym + oth + j] + u[ryp + oth + j])) +
                    (u[r0 + oth + jm] + u[r0 + oth + jp]);
        const T r = f[t] - (s - T(6) * u[t]) / h2;
        const bool cov = in_box(cb, x, y, 2 * (int)j + q);
        if (!cov) acc += (double)r * (double)r;
        if (rout) rout[t] = cov ? R(0) : (R)r;
    }
    return acc;
}

template <class T, class R>
__global__ void k_residual_split(const T* __restrict__ u, const T* __restrict__ f, Lay L, T h2, CovBox cb,
                                 R* __restrict__ rout, double* __restrict__ partials) {
    const double bs = block_sum(body_residual_split<T, R>(u, f, L, h2, cb, rout, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// One outer step of the mixed-precision defect correction on a colour-split periodic level:
//   v   = u_in + (double) e_in          (the pending FP32 correction; e_in == nullptr: none;
//                                        u_in == nullptr: v = 0, the first step of a zero start,
//                                        which then streams f only)
//   r   = f - L v                        (FP64, same arithmetic as k_residual_split)
//   u_out = v,  rhs = (float) r,  e_out = the first red half-sweep of the next inner cycle from
//   e = 0, i.e. (0 - h^2 rhs) / 6 on red cells; black entries are not written.
// v is formed on the fly for the 7 stencil points, so u_out / e_out must not alias the inputs.
// pairs of cells need half-rows of even length (then no pair straddles two half-rows, and the
// 16-byte accesses are aligned)
__host__ __device__ __forceinline__ bool outer_pairs(const Lay& L) { return ((L.d.z >> 1) & 1) == 0; }

// HU: u_in is read (false: a zero start, v = 0); HE: e_in is added.  The three cases are separate
// instantiations: with the choice made per load at run time the kernel measured 193 against
// 167 us at 256^3.
template <bool HU, bool HE, bool WU = HU || HE>
__device__ __forceinline__ double body_outer_split(const double* __restrict__ u_in, const float* __restrict__ e_in,
                                                   const double* __restrict__ f, double* __restrict__ u_out,
                                                   float* __restrict__ rhs, float* __restrict__ e_out,
                                                   const Lay& L, double h2, float h2f, unsigned blk, unsigned nblk) {
    const Dims d = L.d;
    const unsigned n = (unsigned)d.cells();
    double acc = 0.0;
    const RedRange rr = red_range(blk, nblk, (unsigned)n);
    const unsigned lo = rr.lo, hi = rr.hi, stride = rr.stride;
    for (unsigned b0 = lo + threadIdx.x; b0 < hi; b0 += stride)
#pragma unroll
    for (int v = 0; v < kRedV; ++v) {
        const unsigned t = b0 + v * blockDim.x;
        if (t >= hi) break;
        const SplitNb c = split_nb(L, t);
        const unsigned j = c.j, col = c.col, oth = c.oth, r0 = c.r0, rxm = c.rxm, rxp = c.rxp, rym = c.rym,
                       ryp = c.ryp, jm = c.jm, jp = c.jp;
        double c0 = 0.0, s = 0.0;   // a zero start: the stencil sums are +0 exactly
        if constexpr (HU || HE) {
            auto V = [&](unsigned i) {
                if constexpr (HU && HE) return u_in[i] + (double)e_in[i];
                else if constexpr (HU) return u_in[i];
                else return 0.0 + (double)e_in[i];   // u taken as +0 (the same bits as u = +0 read)
            };
            c0 = V(t);
            s = ((V(rxm + oth + j) + V(rxp + oth + j)) + (V(rym + oth + j) + V(ryp + oth + j))) +
                (V(r0 + oth + jm) + V(r0 + oth + jp));
        }
        const double r = f[t] - (s - 6.0 * c0) / h2;
        acc += r * r;
        const float rf = (float)r;
        if constexpr (WU) u_out[t] = c0;   // WU = false: a zero start leaves the zero iterate implicit
        rhs[t] = rf;
        // black entries of e_out are left as they are: the black half-sweep that follows writes
        // every one of them before anything reads them
        if (!col) e_out[t] = (0.0f - h2f * rf) / 6.0f;
    }
    return acc;
}

// The same on pairs of cells: a thread takes the cells t, t + 1 (t even; half-rows have an even
// length here, so both lie in one half-row) and reads every stencil run as a 16-byte u and an
// 8-byte e vector, plus the one z-neighbour entry outside the pair.  Each block covers the same
// cells as in body_outer_split (so batched and solo launches agree); within a block the partial
// sum takes the cells pair by pair.
template <bool HU, bool HE, bool WU = HU || HE>
__device__ __forceinline__ double body_outer_pairs(const double* __restrict__ u_in, const float* __restrict__ e_in,
                                                   const double* __restrict__ f, double* __restrict__ u_out,
                                                   float* __restrict__ rhs, float* __restrict__ e_out,
                                                   const Lay& L, double h2, float h2f, unsigned blk, unsigned nblk) {
    const unsigned n = (unsigned)L.d.cells(), nzh = (unsigned)L.d.z >> 1;
    double acc = 0.0;
    const RedRange rr = red_range(blk, nblk, n);
    const unsigned lo = rr.lo, hi = rr.hi, stride = rr.stride;
    for (unsigned p0 = lo; p0 < hi; p0 += stride)
#pragma unroll
    for (int v = 0; v < kRedV / 2; ++v) {
        const unsigned t = p0 + 2 * (threadIdx.x + v * blockDim.x);
        if (t >= hi) break;
        const SplitNb c = split_nb(L, t);
        const unsigned j = c.j, oth = c.oth, r0 = c.r0, q = (unsigned)c.q;
        // every load of the pair is issued before the first value is formed (a scheduling barrier
        // keeps the compiler from interleaving them with the arithmetic: measured, the waits
        // between groups of loads cost more than the registers the early loads hold)
        const double2 fv = *(const double2*)(f + t);
        double c0[2] = {0.0, 0.0}, s[2] = {0.0, 0.0};   // a zero start: the stencil sums are +0 exactly
        if constexpr (HU || HE) {
            // runs at positions i, i + 1: the cell pair itself, the x and y neighbour rows and the
            // other colour's entries j, j + 1 of this row; then the z-neighbour outside the pair.
            // Cell j + k sits at z = 2(j + k) + q; its z-neighbours are the other colour's entries
            // j + k - 1 + q and j + k + q.
            const unsigned ix[6] = {t, c.rxm + oth + j, c.rxp + oth + j, c.rym + oth + j, c.ryp + oth + j,
                                    r0 + oth + j};
            const unsigned jn = q ? j + 2 : j + nzh - 1;
            const unsigned ie = r0 + oth + (jn >= nzh ? jn - nzh : jn);
            double2 ua[6];
            float2 ea[6];
            double ue = 0.0;
            float ee = 0.0f;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                if constexpr (HU) ua[k] = *(const double2*)(u_in + ix[k]);
                if constexpr (HE) ea[k] = *(const float2*)(e_in + ix[k]);
            }
            if constexpr (HU) ue = u_in[ie];
            if constexpr (HE) ee = e_in[ie];
            __builtin_amdgcn_sched_barrier(0);
            // v = u (+ e), u taken as +0 without HU (the same bits as u = +0 read)
            auto V = [&](double a, float b) {
                if constexpr (HU && HE) return a + (double)b;
                else if constexpr (HU) return a;
                else return 0.0 + (double)b;
            };
            double w[6][2];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                w[k][0] = V(HU ? ua[k].x : 0.0, HE ? ea[k].x : 0.0f);
                w[k][1] = V(HU ? ua[k].y : 0.0, HE ? ea[k].y : 0.0f);
            }
            const double edge = V(ue, ee);
            c0[0] = w[0][0];
            c0[1] = w[0][1];
            const double* cz = w[5];
            const double zm0 = q ? cz[0] : edge, zp0 = q ? cz[1] : cz[0];
            const double zm1 = q ? cz[1] : cz[0], zp1 = q ? edge : cz[1];
            s[0] = ((w[1][0] + w[2][0]) + (w[3][0] + w[4][0])) + (zm0 + zp0);
            s[1] = ((w[1][1] + w[2][1]) + (w[3][1] + w[4][1])) + (zm1 + zp1);
        }
        const double r0v = fv.x - (s[0] - 6.0 * c0[0]) / h2;
        const double r1v = fv.y - (s[1] - 6.0 * c0[1]) / h2;
        acc += r0v * r0v;
        acc += r1v * r1v;
        const float rf0 = (float)r0v, rf1 = (float)r1v;
        if constexpr (WU) *(double2*)(u_out + t) = double2{c0[0], c0[1]};
        *(float2*)(rhs + t) = float2{rf0, rf1};
        // black entries of e_out are left as they are (see body_outer_split)
        if (!c.col) *(float2*)(e_out + t) = float2{(0.0f - h2f * rf0) / 6.0f, (0.0f - h2f * rf1) / 6.0f};
    }
    return acc;
}

__device__ __forceinline__ double body_outer_split_any(const double* __restrict__ u_in,
                                                       const float* __restrict__ e_in, const double* __restrict__ f,
                                                       double* __restrict__ u_out, float* __restrict__ rhs,
                                                       float* __restrict__ e_out, const Lay& L, double h2, float h2f,
                                                       unsigned blk, unsigned nblk) {
    if (outer_pairs(L)) {
        if (!u_in) return body_outer_pairs<false, false, true>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blk, nblk);
        if (e_in) return body_outer_pairs<true, true>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blk, nblk);
        return body_outer_pairs<true, false>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blk, nblk);
    }
    if (!u_in) return body_outer_split<false, false, true>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blk, nblk);
    if (e_in) return body_outer_split<true, true>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blk, nblk);
    return body_outer_split<true, false>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blk, nblk);
}

template <bool HU, bool HE, bool WU>
__global__ void k_outer_pairs(const double* __restrict__ u_in, const float* __restrict__ e_in,
                              const double* __restrict__ f, double* __restrict__ u_out, float* __restrict__ rhs,
                              float* __restrict__ e_out, Lay L, double h2, float h2f,
                              double* __restrict__ partials) {
    const double bs =
        block_sum(body_outer_pairs<HU, HE, WU>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

template <bool HU, bool HE, bool WU>
__global__ void k_outer_split(const double* __restrict__ u_in, const float* __restrict__ e_in,
                              const double* __restrict__ f, double* __restrict__ u_out, float* __restrict__ rhs,
                              float* __restrict__ e_out, Lay L, double h2, float h2f,
                              double* __restrict__ partials) {
    const double bs =
        block_sum(body_outer_split<HU, HE, WU>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

void launch_outer_split(const double* u_in, const float* e_in, const double* f, double* u_out, float* rhs,
                        float* e_out, Lay L, double h, double* partials, int* nparts, hipStream_t st) {
    const int g = grid_for(L.d.cells(), kBlock * kRedV, kMaxPartials);
    const double h2 = h * h;
    const float h2f = (float)(h * h);
#define MG_OUTER(K, HU, HE) K<HU, HE, HU || HE><<<g, kBlock, 0, st>>>(u_in, e_in, f, u_out, rhs, e_out, L, h2, h2f, partials)
    if (outer_pairs(L)) {
        if (u_in && e_in) MG_OUTER(k_outer_pairs, true, true);
        else if (u_in) MG_OUTER(k_outer_pairs, true, false);
        else if (e_in) MG_OUTER(k_outer_pairs, false, true);
        else MG_OUTER(k_outer_pairs, false, false);
    } else {
        if (u_in && e_in) MG_OUTER(k_outer_split, true, true);
        else if (u_in) MG_OUTER(k_outer_split, true, false);
        else if (e_in) MG_OUTER(k_outer_split, false, true);
        else MG_OUTER(k_outer_split, false, false);
    }
#undef MG_OUTER
    *nparts = g;
}

__device__ __forceinline__ double body_sum(const double* __restrict__ a, const Lay& L, const CovBox& cb, int square,
                                           unsigned blk, unsigned nblk) {
    double acc = 0.0;
    const size_t n = L.d.cells();
    const unsigned lo = red_lo(blk), hi = (unsigned)n, stride = red_stride(nblk);
    for (unsigned b0 = lo + threadIdx.x; b0 < hi; b0 += stride)
#pragma unroll
    for (int v = 0; v < kRedV; ++v) {
        const unsigned i = b0 + v * blockDim.x;
        if (i >= hi) break;
        int x, y, z;
        ldecode(L, i, x, y, z);
        if (in_box(cb, x, y, z)) continue;
        const double av = a[i];
        acc += square ? av * av : av;
    }
    return acc;
}

__global__ void k_sum(const double* __restrict__ a, Lay L, CovBox cb, int square, double* __restrict__ partials) {
    const double bs = block_sum(body_sum(a, L, cb, square, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// Fused passes of the source preparation and of the final gauge on a level (natural user rows
// <-> the level's layout).  The reductions stride exactly like body_sum over the level array, so
// their partial sums have the same bits as a separate copy followed by body_sum.
// dst (layout L) = src (natural rows); partial sums of the copied values
__device__ __forceinline__ double body_relayout_sum(const double* __restrict__ src, double* __restrict__ dst,
                                                    const Lay& L, unsigned blk, unsigned nblk) {
    double acc = 0.0;
    const unsigned n = (unsigned)L.d.cells();
    const unsigned lo = red_lo(blk), stride = red_stride(nblk);
    for (unsigned b0 = lo + threadIdx.x; b0 < n; b0 += stride)
#pragma unroll
    for (int v = 0; v < kRedV; ++v) {
        const unsigned i = b0 + v * blockDim.x;
        if (i >= n) break;
        int x, y, z;
        ldecode(L, i, x, y, z);
        const double av = src[lidx(L.d, 0, x, y, z)];
        dst[i] = av;
        acc += av;
    }
    return acc;
}
// a -= sum * inv (as k_sub_mean); partial sums of the new values squared
__device__ __forceinline__ double body_submean_sumsq(double* __restrict__ a, const Lay& L,
                                                     const double* __restrict__ sum, double inv, unsigned blk,
                                                     unsigned nblk) {
    const double m = sum[0] * inv;
    double acc = 0.0;
    const unsigned n = (unsigned)L.d.cells();
    const unsigned lo = red_lo(blk), stride = red_stride(nblk);
    for (unsigned b0 = lo + threadIdx.x; b0 < n; b0 += stride)
#pragma unroll
    for (int v = 0; v < kRedV; ++v) {
        const unsigned i = b0 + v * blockDim.x;
        if (i >= n) break;
        const double av = a[i] - m;
        a[i] = av;
        acc += av * av;
    }
    return acc;
}

__global__ void k_relayout_sum(const double* __restrict__ src, double* __restrict__ dst, Lay L,
                               double* __restrict__ partials) {
    const double bs = block_sum(body_relayout_sum(src, dst, L, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}
__global__ void k_submean_sumsq(double* __restrict__ a, Lay L, const double* __restrict__ sum, double inv,
                                double* __restrict__ partials) {
    const double bs = block_sum(body_submean_sumsq(a, L, sum, inv, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}
// dst (layout LD) = src (layout LS) - sum * inv: the copy back of the gauge's mean removal
__global__ void k_relayout_sub(const double* __restrict__ src, Lay LS, double* __restrict__ dst, Lay LD,
                               const double* __restrict__ sum, double inv) {
    const double m = sum[0] * inv;
    const size_t n = LD.d.cells();
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        ldecode(LD, i, x, y, z);
        dst[i] = src[lidx(LS, x, y, z)] - m;
    }
}

// w * sum(partials[0..cnt)), added to total on thread 0, in a fixed order
__device__ __forceinline__ void body_finalize_seg(const double* __restrict__ partials, int cnt, double w,
                                                  double& total) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) acc += partials[i];
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) total += w * bs;
}

__global__ void k_finalize(const double* __restrict__ partials, SegList segs, double* __restrict__ out) {
    double total = 0.0;
    for (int s = 0; s < segs.n; ++s) body_finalize_seg(partials + segs.off[s], segs.cnt[s], segs.w[s], total);
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
void launch_relayout(const A* src, Lay ls, B* dst, Lay ld, hipStream_t st) {
    k_relayout<A, B><<<grid_for(ld.d.cells(), kBlock, 8192), kBlock, 0, st>>>(src, ls, dst, ld);
}
void launch_add_f32_to_f64(double* u, const float* e, size_t n, hipStream_t st) {
    k_add_f32<<<grid_for(n, kBlock, 8192), kBlock, 0, st>>>(u, e, n);
}
template <class T>
void launch_sub_mean(T* a, size_t n, const double* sum, double inv_count, hipStream_t st) {
    k_sub_mean<T><<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(a, n, sum, inv_count);
}

template <class T>
void launch_rbgs_half(T* u, const T* f, const T* ghosts, Lay L, double h, int colour, hipStream_t st,
                      hipEvent_t ev0, hipEvent_t ev1) {
    const size_t n = (size_t)L.d.x * L.d.y * (L.d.z / 2);
    const T h2 = (T)(h * h);
    // stamped by the events when they are given (kernel timing), else a plain launch (the form
    // captured into graphs)
    constexpr int W = Vec16<T>::W;
    const bool vec = (L.d.z / 2) % W == 0 && (((uintptr_t)u | (uintptr_t)f) & 15u) == 0;
    if (ghosts && vec) {   // runs of W cells (same bits)
        const unsigned g = grid_for(n / W);
        if (ev0)
            hipExtLaunchKernelGGL(k_rbgs_ghost_vec<T>, dim3(g), dim3(kBlock), 0, st, ev0, ev1, 0, u, f, ghosts, L, h2,
                                  colour);
        else
            k_rbgs_ghost_vec<T><<<g, kBlock, 0, st>>>(u, f, ghosts, L, h2, colour);
    } else if (ghosts) {
        if (ev0)
            hipExtLaunchKernelGGL(k_rbgs_ghost<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, ev0, ev1, 0, u, f, ghosts,
                                  L, h2, colour);
        else
            k_rbgs_ghost<T><<<grid_for(n), kBlock, 0, st>>>(u, f, ghosts, L, h2, colour);
    } else if (sizeof(T) == 4 && n >= ((size_t)1 << 22)) {   // measured: 4 cells per thread for FP32 at 256^3+
        const unsigned g = rbgs_split_blocks(L, kBlock, 4);
        if (ev0)
            hipExtLaunchKernelGGL(k_rbgs_split<T, 4>, dim3(g), dim3(kBlock), 0, st, ev0, ev1, 0, u, f, L, h2, colour);
        else
            k_rbgs_split<T, 4><<<g, kBlock, 0, st>>>(u, f, L, h2, colour);
    } else if (n >= (size_t)kBlock * 64 * 2) {
        const unsigned g = rbgs_split_blocks(L, kBlock, 2);
        if (ev0)
            hipExtLaunchKernelGGL(k_rbgs_split<T, 2>, dim3(g), dim3(kBlock), 0, st, ev0, ev1, 0, u, f, L, h2, colour);
        else
            k_rbgs_split<T, 2><<<g, kBlock, 0, st>>>(u, f, L, h2, colour);
    } else {
        const unsigned g = rbgs_split_blocks(L, kBlock, 1);
        if (ev0)
            hipExtLaunchKernelGGL(k_rbgs_split<T, 1>, dim3(g), dim3(kBlock), 0, st, ev0, ev1, 0, u, f, L, h2, colour);
        else
            k_rbgs_split<T, 1><<<g, kBlock, 0, st>>>(u, f, L, h2, colour);
    }
}

// dynamic LDS above the default for the tail kernels; set once, before any graph capture
hipError_t tail_kernel_setup() {
    static bool done = false;
    if (done) return hipSuccess;
    const void* fns[4] = {(const void*)k_tail<float>, (const void*)k_tail<double>, (const void*)k_tail_p2<float>,
                          (const void*)k_tail_p2<double>};
    for (const void* fn : fns) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTailMaxLds);
        if (e != hipSuccess) return e;
    }
    done = true;
    return hipSuccess;
}

template <class T>
void launch_tail(const TailPlan<T>& tp, hipStream_t st) {
    (void)tail_kernel_setup();
    bool p2 = tp.n >= 2 && tp.lev[tp.n - 1].lay.d.cells() == 1;
    for (int k = 0; p2 && k + 1 < tp.n; ++k) {
        const Lay& A = tp.lev[k].lay;
        p2 = A.pow2 && A.split && A.d.x == A.d.y && A.d.y == A.d.z && A.lgx == tp.lev[0].lay.lgx - k;
    }
    if (p2) k_tail_p2<T><<<1, kTailThreads, tp.lds_bytes, st>>>(tp);
    else k_tail<T><<<1, kTailThreads, tp.lds_bytes, st>>>(tp);
}

template <class T>
void launch_resid_restrict(const T* u, const T* f, const T* ghosts, Lay L, double h, T* pu, T* pf, T* uold,
                           ParentMap pm, hipStream_t st) {
    const Lay C = mklay(Dims{L.d.x / 2, L.d.y / 2, L.d.z / 2}, 0);
    const size_t n = C.d.cells();
    const T h2 = (T)(h * h);
    if (ghosts && L.split)   // colour-split patch: all loads of a coarse cell issued at once (same bits)
        k_resid_restrict_gh<T><<<grid_for(n), kBlock, 0, st>>>(u, f, ghosts, L, h2, pu, pf, uold, pm, C);
    else if (ghosts)
        k_resid_restrict<T, true><<<grid_for(n), kBlock, 0, st>>>(u, f, ghosts, L, h2, pu, pf, uold, pm, C);
    else
        k_resid_restrict<T, false><<<grid_for(n), kBlock, 0, st>>>(u, f, nullptr, L, h2, pu, pf, uold, pm, C);
}

template <class T>
void launch_fas_rhs(const T* pu, T* pf, ParentMap pm, Dims cov, double H, hipStream_t st) {
    k_fas_rhs<T><<<grid_for(cov.cells()), kBlock, 0, st>>>(pu, pf, pm, mklay(cov, 0), (T)(H * H));
}

template <class T>
void launch_prolong(T* u, Lay L, const T* pu, const T* uold, ParentMap pm, int black_only, hipStream_t st) {
    if (black_only && L.split)
        k_prolong_black<T><<<grid_for(L.d.cells() >> 1), kBlock, 0, st>>>(u, L, pu, uold, pm);
    else
        k_prolong<T><<<grid_for(L.d.cells()), kBlock, 0, st>>>(u, L, pu, uold, pm);
}

template <class T>
void launch_coarsest(T* u, const T* f, int M, double h, hipStream_t st) {
    k_coarsest<T><<<1, kBlock, 0, st>>>(u, f, M, h);
}

template <class T>
void launch_ghost_fill(const T* pu, const T* u, T* ghosts, Lay L, ParentMap pm, int flux_match, hipStream_t st,
                       double* part, int mode) {
    const Dims d = L.d;
    const size_t most = std::max({(size_t)(d.y / 2) * (d.z / 2), (size_t)(d.x / 2) * (d.z / 2),
                                  (size_t)(d.x / 2) * (d.y / 2)});
    const dim3 grid(grid_for(4 * most), 6);
    double2* pa = (double2*)part;
    if (!pa || mode == 0) k_ghost_fill<T, 0><<<grid, kBlock, 0, st>>>(pu, u, ghosts, nullptr, L, pm, flux_match);
    else if (mode == 1) k_ghost_fill<T, 1><<<grid, kBlock, 0, st>>>(pu, u, ghosts, pa, L, pm, flux_match);
    else k_ghost_fill<T, 2><<<grid, kBlock, 0, st>>>(pu, u, ghosts, pa, L, pm, flux_match);
}

template <class T>
void launch_restrict_cov(const T* fine, Lay L, T* parent, ParentMap pm, hipStream_t st) {
    const size_t n = (size_t)(L.d.x / 2) * (L.d.y / 2) * (L.d.z / 2);
    k_restrict_cov<T><<<grid_for(n), kBlock, 0, st>>>(fine, L, parent, pm);
}

template <class T, class R>
void launch_residual(const T* u, const T* f, const T* ghosts, Lay L, double h, CovBox cov, R* rout, Lay LR,
                     double* partials, int* nparts, hipStream_t st) {
    const int g = grid_for(L.d.cells(), kBlock * kRedV, kMaxPartials);
    const T h2 = (T)(h * h);
    if (ghosts)
        k_residual<T, R, true><<<g, kBlock, 0, st>>>(u, f, ghosts, L, h2, cov, rout, LR, partials);
    else if (L.split && (!rout || LR.split))
        k_residual_split<T, R><<<g, kBlock, 0, st>>>(u, f, L, h2, cov, rout, partials);
    else
        k_residual<T, R, false><<<g, kBlock, 0, st>>>(u, f, nullptr, L, h2, cov, rout, LR, partials);
    *nparts = g;
}

void launch_sum(const double* a, Lay L, CovBox cov, int square, double* partials, int* nparts, hipStream_t st) {
    const int g = grid_for(L.d.cells(), kBlock * kRedV, kMaxPartials);
    k_sum<<<g, kBlock, 0, st>>>(a, L, cov, square, partials);
    *nparts = g;
}

void launch_relayout_sum(const double* src, double* dst, Lay L, double* partials, int* nparts, hipStream_t st) {
    const int g = grid_for(L.d.cells(), kBlock * kRedV, kMaxPartials);
    k_relayout_sum<<<g, kBlock, 0, st>>>(src, dst, L, partials);
    *nparts = g;
}
void launch_submean_sumsq(double* a, Lay L, const double* sum, double inv, double* partials, int* nparts,
                          hipStream_t st) {
    const int g = grid_for(L.d.cells(), kBlock * kRedV, kMaxPartials);
    k_submean_sumsq<<<g, kBlock, 0, st>>>(a, L, sum, inv, partials);
    *nparts = g;
}
void launch_relayout_sub(const double* src, Lay ls, double* dst, Lay ld, const double* sum, double inv,
                         hipStream_t st) {
    k_relayout_sub<<<grid_for(ld.d.cells(), kBlock, 8192), kBlock, 0, st>>>(src, ls, dst, ld, sum, inv);
}

void launch_finalize(const double* partials, SegList segs, double* out, hipStream_t st) {
    k_finalize<<<1, kBlock, 0, st>>>(partials, segs, out);
}

// ----------------------------------------------------------------------------------------------
// batched kernels: one launch covers the same step of many independent instances.  A block
// finds its instance by binary search over the segment table (block-uniform, so scalar loads)
// and then runs the plain kernel's body with its block index inside the instance.
// ----------------------------------------------------------------------------------------------

// A whole periodic colour-split power-of-two cube whose half-rows hold whole runs of W cells
// (16 bytes): its FAS right-hand side and black prolongation take the run bodies.
__host__ __device__ inline bool p2_runs(const Lay& L, unsigned W) {
    return L.pow2 && L.split && L.lgx == L.lgy && L.lgy == L.lgz && L.lgz >= 2 && ((1u << (L.lgz - 1)) % W) == 0;
}
__host__ __device__ inline bool whole_periodic(const ParentMap& pm) {
    return pm.periodic && pm.off[0] == 0 && pm.off[1] == 0 && pm.off[2] == 0;
}
// FAS on the covered box C of parent pm: the whole parent
__host__ __device__ inline bool fas_runs(const Lay& C, const ParentMap& pm, unsigned W) {
    return p2_runs(pm.pl, W) && whole_periodic(pm) && C.d.x == pm.pl.d.x && C.d.y == pm.pl.d.y && C.d.z == pm.pl.d.z;
}
// black prolongation of level L from its whole coarsening pm
__host__ __device__ inline bool prolong_runs(const Lay& L, const ParentMap& pm, unsigned W) {
    return p2_runs(L, W) && pm.pl.pow2 && pm.pl.split && whole_periodic(pm) && pm.pl.lgx == L.lgx - 1 &&
           pm.pl.lgy == L.lgy - 1 && pm.pl.lgz == L.lgz - 1;
}
// blocks of kBlock threads for a batched FAS / black-prolongation segment
unsigned fas_blocks(const Lay& C, const ParentMap& pm, int elem) {
    const unsigned W = 16u / (unsigned)elem;
    const size_t n = fas_runs(C, pm, W) ? C.d.cells() / 2 / W : C.d.cells();
    return (unsigned)((n + kBlock - 1) / kBlock);
}
unsigned prolong_black_blocks(const Lay& L, const ParentMap& pm, int elem) {
    const unsigned W = 16u / (unsigned)elem;
    const size_t n = prolong_runs(L, pm, W) ? L.d.cells() / 2 / W : L.d.cells() / 2;
    return (unsigned)((n + kBlock - 1) / kBlock);
}

__device__ __forceinline__ const BSeg& seg_of(const BSeg* __restrict__ segs, int nseg, unsigned& lb) {
    const unsigned b = blockIdx.x;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    lb = b - segs[lo].blk0;
    return segs[lo];
}

template <class T, int V>
__global__ void kb_rbgs(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active, int colour) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L;
    // with V = W cells per thread a block covers the same cells as a block of 16-byte runs, so
    // the power-of-two levels whose half-rows hold whole runs take the 16-byte body (same bits)
    if constexpr (V == Vec16<T>::W) {
        if (L.pow2 && L.split && L.lgz >= 1 && ((1u << (L.lgz - 1)) % V) == 0) {
            const unsigned ch = lb * blockDim.x + threadIdx.x;
            if (ch < (unsigned)(L.d.cells() / 2 / V))
                run_rbgs_vec<T>((T*)s.a[0], (const T*)s.a[1], L.lgx, L.lgy, L.lgz, (T)(s.h * s.h), colour, ch);
            return;
        }
    }
    body_rbgs_split<T, V>((T*)s.a[0], (const T*)s.a[1], L, (T)(s.h * s.h), colour, lb);
}

template <class T>
__global__ void kb_resid_restrict(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L, C = s.C;
    const ParentMap pm = s.pm;
    const unsigned t = lb * blockDim.x + threadIdx.x;
    if (t >= (unsigned)C.d.cells()) return;
    // a whole power-of-two cube with a colour-split parent: the power-of-two body (one thread per
    // coarse cell in natural order, as here; same bits)
    if (L.pow2 && L.split && pm.pl.split && L.d.x == L.d.y && L.d.y == L.d.z && L.d.x >= 4 && pm.periodic &&
        pm.off[0] == 0 && pm.off[1] == 0 && pm.off[2] == 0) {
        cell_resid_restrict_p2<T>((const T*)s.a[0], (const T*)s.a[1], L.lgx, (T)(s.h * s.h), (T*)s.a[2], (T*)s.a[3],
                                  (T*)s.a[4], t);
        return;
    }
    cell_resid_restrict<T, false>((const T*)s.a[0], (const T*)s.a[1], nullptr, L, (T)(s.h * s.h), (T*)s.a[2],
                                  (T*)s.a[3], (T*)s.a[4], pm, C, t);
}

template <class T>
__global__ void kb_fas(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay C = s.C;
    const ParentMap pm = s.pm;
    const unsigned t = lb * blockDim.x + threadIdx.x;
    if (fas_runs(C, pm, Vec16<T>::W)) {   // 16-byte runs of both colours (same bits)
        if (t < (unsigned)(C.d.cells() / 2 / Vec16<T>::W)) run_fas_vec<T>((const T*)s.a[0], (T*)s.a[1], pm.pl.lgx, (T)(s.h * s.h), t);
        return;
    }
    if (t < (unsigned)C.d.cells()) cell_fas<T>((const T*)s.a[0], (T*)s.a[1], pm, C, (T)(s.h * s.h), t);
}

template <class T, bool BLACK>
__global__ void kb_prolong(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L;
    const ParentMap pm = s.pm;
    const unsigned t = lb * blockDim.x + threadIdx.x;
    if constexpr (BLACK) {
        if (prolong_runs(L, pm, Vec16<T>::W)) {   // 16-byte runs of black cells (same bits)
            if (t < (unsigned)(L.d.cells() / 2 / Vec16<T>::W))
                run_prolong_black_vec<T>((T*)s.a[0], L.lgx, (const T*)s.a[1], (const T*)s.a[2], t);
            return;
        }
        if (t < (unsigned)(L.d.cells() >> 1))
            cell_prolong_black<T>((T*)s.a[0], L, (const T*)s.a[1], (const T*)s.a[2], pm, t);
    } else {
        if (t < (unsigned)L.d.cells()) cell_prolong<T>((T*)s.a[0], L, (const T*)s.a[1], (const T*)s.a[2], pm, t);
    }
}

// Each workgroup first copies its plan into LDS and body_tail marks every field it takes from
// the plan as wave-uniform (read from global memory with a run-time level index, the plan was
// pulled into vector registers and spilled; this way a few words still spill on FP64).
template <class T>
__global__ void __launch_bounds__(kTailThreads) kb_tail(const TailPlan<T>* __restrict__ plans,
                                                        const int* __restrict__ active) {
    __shared__ __align__(16) unsigned char raw[sizeof(TailPlan<T>)];
    static_assert(sizeof(TailPlan<T>) % 4 == 0, "plan copied as 32-bit words");
    const unsigned* src = (const unsigned*)(plans + blockIdx.x);
    for (unsigned w = threadIdx.x; w < sizeof(TailPlan<T>) / 4; w += blockDim.x) ((unsigned*)raw)[w] = src[w];
    __syncthreads();
    const TailPlan<T>& sp = *reinterpret_cast<const TailPlan<T>*>(raw);
    if (!active[uniform(sp.inst)]) return;
    body_tail<T>(sp);
}

__global__ void kb_outer(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active, int has_e,
                         int zero_u) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L;
    const double acc = body_outer_split_any(zero_u ? nullptr : (const double*)s.a[0], has_e ? (const float*)s.a[1] : nullptr,
                                        (const double*)s.a[2], (double*)s.a[3], (float*)s.a[4], (float*)s.a[5], L,
                                        s.h * s.h, (float)(s.h * s.h), lb, s.nblk);
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) s.part[lb] = bs;
}

__global__ void kb_residual(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L;
    const CovBox none{};
    const double acc = body_residual_split<double, double>((const double*)s.a[0], (const double*)s.a[1], L,
                                                           s.h * s.h, none, nullptr, lb, s.nblk);
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) s.part[lb] = bs;
}

__global__ void kb_sum(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active, int square) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L;
    const CovBox none{};
    const double bs = block_sum(body_sum((const double*)s.a[0], L, none, square, lb, s.nblk));
    if (threadIdx.x == 0) s.part[lb] = bs;
}

__global__ void kb_finalize(const BFin* __restrict__ fins, const int* __restrict__ active) {
    if (!active[blockIdx.x]) return;
    const BFin& f = fins[blockIdx.x];
    double total = 0.0;
    body_finalize_seg(f.part, f.cnt, f.w, total);
    if (threadIdx.x == 0) f.out[0] = total;
}

// a = {src (natural rows), dst (layout L)}: the copy-in with its sum
__global__ void kb_relayout_sum(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L;
    const double bs = block_sum(body_relayout_sum((const double*)s.a[0], (double*)s.a[1], L, lb, s.nblk));
    if (threadIdx.x == 0) s.part[lb] = bs;
}
// a = {array (layout L), sum}, h = 1 / cells: mean removal with the sum of squares
__global__ void kb_submean_sumsq(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay L = s.L;
    const double bs = block_sum(body_submean_sumsq((double*)s.a[0], L, (const double*)s.a[1], s.h, lb, s.nblk));
    if (threadIdx.x == 0) s.part[lb] = bs;
}

// grid-stride loops over one instance's cells with its own blocks
__global__ void kb_sub_mean(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    double* a = (double*)s.a[0];
    const double m = ((const double*)s.a[1])[0] * s.h;
    const size_t n = s.L.d.cells();
    for (size_t i = lb * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)s.nblk * blockDim.x) a[i] = a[i] - m;
}

// a = {src (layout L), dst (layout C), sum}, h = 1 / cells: the copy back with the mean removed
__global__ void kb_relayout_sub(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay ls = s.L, ld = s.C;
    const double* src = (const double*)s.a[0];
    double* dst = (double*)s.a[1];
    const double m = ((const double*)s.a[2])[0] * s.h;
    const size_t n = ld.d.cells();
    for (size_t i = lb * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)s.nblk * blockDim.x) {
        int x, y, z;
        ldecode(ld, i, x, y, z);
        dst[i] = src[lidx(ls, x, y, z)] - m;
    }
}

__global__ void kb_relayout(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    const Lay ls = s.L, ld = s.C;
    const double* src = (const double*)s.a[0];
    double* dst = (double*)s.a[1];
    const size_t n = ld.d.cells();
    for (size_t i = lb * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)s.nblk * blockDim.x) {
        int x, y, z;
        ldecode(ld, i, x, y, z);
        dst[i] = src[lidx(ls, x, y, z)];
    }
}

template <class T>
__global__ void kb_zero(const BSeg* __restrict__ segs, int nseg, const int* __restrict__ active) {
    unsigned lb;
    const BSeg& s = seg_of(segs, nseg, lb);
    if (!active[s.inst]) return;
    T* p = (T*)s.a[0];
    const size_t n = s.L.d.cells();
    for (size_t i = lb * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)s.nblk * blockDim.x) p[i] = T(0);
}

template <class T>
void launch_b_rbgs(const BSeg* segs, int nseg, unsigned grid, int block, int V, const int* active, int colour,
                   hipStream_t st) {
    switch (V) {
        case 1: kb_rbgs<T, 1><<<grid, block, 0, st>>>(segs, nseg, active, colour); break;
        case 2: kb_rbgs<T, 2><<<grid, block, 0, st>>>(segs, nseg, active, colour); break;
        default: kb_rbgs<T, 4><<<grid, block, 0, st>>>(segs, nseg, active, colour); break;
    }
}
template <class T>
void launch_b_resid_restrict(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_resid_restrict<T><<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
template <class T>
void launch_b_fas(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_fas<T><<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
template <class T>
void launch_b_prolong(const BSeg* segs, int nseg, unsigned grid, const int* active, int black_only, hipStream_t st) {
    if (black_only) kb_prolong<T, true><<<grid, kBlock, 0, st>>>(segs, nseg, active);
    else kb_prolong<T, false><<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
hipError_t batch_kernel_setup() {
    static bool done = false;
    if (done) return hipSuccess;
    // kb_tail holds its plan in static LDS besides the dynamic levels; it asks for the bound on
    // what a tail plan needs, not for the whole workgroup LDS
    hipError_t e = hipFuncSetAttribute((const void*)kb_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kTailLdsBound);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)kb_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kTailLdsBound);
    if (e == hipSuccess) done = true;
    return e;
}
template <class T>
void launch_b_tail(const TailPlan<T>* plans, int n, unsigned lds_bytes, const int* active, hipStream_t st) {
    kb_tail<T><<<n, kTailThreads, lds_bytes, st>>>(plans, active);
}
void launch_b_outer(const BSeg* segs, int nseg, unsigned grid, const int* active, int has_e, int zero_u,
                    hipStream_t st) {
    kb_outer<<<grid, kBlock, 0, st>>>(segs, nseg, active, has_e, zero_u);
}
void launch_b_residual(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_residual<<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
void launch_b_sum(const BSeg* segs, int nseg, unsigned grid, const int* active, int square, hipStream_t st) {
    kb_sum<<<grid, kBlock, 0, st>>>(segs, nseg, active, square);
}
void launch_b_finalize(const BFin* fins, int n, const int* active, hipStream_t st) {
    kb_finalize<<<n, kBlock, 0, st>>>(fins, active);
}
void launch_b_sub_mean(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_sub_mean<<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
void launch_b_relayout_sum(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_relayout_sum<<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
void launch_b_submean_sumsq(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_submean_sumsq<<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
void launch_b_relayout_sub(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_relayout_sub<<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
void launch_b_relayout(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_relayout<<<grid, kBlock, 0, st>>>(segs, nseg, active);
}
template <class T>
void launch_b_zero(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st) {
    kb_zero<T><<<grid, kBlock, 0, st>>>(segs, nseg, active);
}

// explicit instantiations
template void launch_fill<double>(double*, size_t, double, hipStream_t);
template void launch_fill<float>(float*, size_t, float, hipStream_t);
template void launch_relayout<double, float>(const double*, Lay, float*, Lay, hipStream_t);
template void launch_relayout<float, double>(const float*, Lay, double*, Lay, hipStream_t);
template void launch_relayout<double, double>(const double*, Lay, double*, Lay, hipStream_t);
template void launch_sub_mean<double>(double*, size_t, const double*, double, hipStream_t);
#define MGIC_INST(T)                                                                                        \
    template void launch_rbgs_half<T>(T*, const T*, const T*, Lay, double, int, hipStream_t, hipEvent_t,      \
                                      hipEvent_t);               \
    template void launch_resid_restrict<T>(const T*, const T*, const T*, Lay, double, T*, T*, T*, ParentMap, \
                                           hipStream_t);                                                    \
    template void launch_fas_rhs<T>(const T*, T*, ParentMap, Dims, double, hipStream_t);                    \
    template void launch_prolong<T>(T*, Lay, const T*, const T*, ParentMap, int, hipStream_t);                   \
    template void launch_coarsest<T>(T*, const T*, int, double, hipStream_t);                               \
    template void launch_ghost_fill<T>(const T*, const T*, T*, Lay, ParentMap, int, hipStream_t, double*, int); \
    template void launch_restrict_cov<T>(const T*, Lay, T*, ParentMap, hipStream_t);                \
    template void launch_tail<T>(const TailPlan<T>&, hipStream_t);
MGIC_INST(double)
MGIC_INST(float)
#undef MGIC_INST
#define MGIC_BINST(T)                                                                                         \
    template void launch_b_rbgs<T>(const BSeg*, int, unsigned, int, int, const int*, int, hipStream_t);         \
    template void launch_b_resid_restrict<T>(const BSeg*, int, unsigned, const int*, hipStream_t);             \
    template void launch_b_fas<T>(const BSeg*, int, unsigned, const int*, hipStream_t);                        \
    template void launch_b_prolong<T>(const BSeg*, int, unsigned, const int*, int, hipStream_t);               \
    template void launch_b_tail<T>(const TailPlan<T>*, int, unsigned, const int*, hipStream_t);                \
    template void launch_b_zero<T>(const BSeg*, int, unsigned, const int*, hipStream_t);
MGIC_BINST(double)
MGIC_BINST(float)
#undef MGIC_BINST
template void launch_residual<double, double>(const double*, const double*, const double*, Lay, double, CovBox,
                                              double*, Lay, double*, int*, hipStream_t);
template void launch_residual<double, float>(const double*, const double*, const double*, Lay, double, CovBox,
                                             float*, Lay, double*, int*, hipStream_t);

}  // namespace mgic
