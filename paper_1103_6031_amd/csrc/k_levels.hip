// Fused small-level kernels of the FAS V-cycle (Section 3.2) for the periodic coarsenings that
// are power-of-two cubes of 16^3, 32^3 and 64^3 cells.
//
// As one-step kernels each such level costs eleven launches per cycle (FAS right-hand side,
// 2 nu1 half-sweeps, residual + restriction, prolongation, 2 nu2 half-sweeps), and at these sizes
// every launch costs about its dispatch latency.  Here one workgroup per 8^3 tile holds the tile
// and a halo in LDS and runs a whole leg of the cycle there:
//   pre:  FAS right-hand side (step 6 of the parent), nu1 red-black sweeps (step 2), residual and
//         restriction (steps 3-5) of the tile;
//   post: coarse-grid correction (step 8), nu2 red-black sweeps (step 9) of the tile.
// A half-sweep of a cell needs its neighbours' previous values, so after each half-sweep the
// region that is still exact shrinks by one cell; the halo is as deep as the number of
// half-sweeps (plus one for the residual stencil), and the halo cells are computed redundantly
// by the neighbouring tiles.  Every value is formed by the same operations in the same order as
// in the one-step kernels, so the results are bit-identical to them.  Workgroups read the level's
// arrays and write a second copy (no workgroup reads what another writes).

#include <hip/hip_ext.h>

#include "mg_internal.h"
#include "p2_bodies.h"

namespace mgic {

constexpr int kTile = 8;            // tile edge (cells)
constexpr int kFusedThreads = 512;  // one thread per tile cell

// Loops over the cells of a region: each thread takes the cells t = threadIdx.x + r * 512; every
// pass first forms all its values (an index past the end is clamped to the last cell, so every
// load stays inside the arrays) and only then stores them, so that the loads of all passes are in
// flight together.
template <int N>
struct Passes {
    static constexpr int n = (N + kFusedThreads - 1) / kFusedThreads;
    __device__ static int cell(int r) {
        const int t = (int)threadIdx.x + r * kFusedThreads;
        return t < N ? t : N - 1;
    }
    __device__ static bool live(int r) { return N % kFusedThreads == 0 || (int)threadIdx.x + r * kFusedThreads < N; }
};

// one red-black half-sweep of `colour` over the cells of [k, S - k)^3 of an S^3 LDS region of u
// (origin parity p0: the cell (i, j, m) has colour (i + j + m + p0) & 1); f is the (S - 2)^3
// region one cell inside it.  The cells of one colour read only the other colour, so all new
// values are formed before any is stored.
template <class T, int S, int k>
__device__ __forceinline__ void lds_half_sweep(T* su, const T* sf, T h2, int colour, int p0) {
    constexpr int W = S - 2 * k, Wh = W / 2, SF = S - 2;
    using Pp = Passes<W * W * Wh>;
    T v[Pp::n];
    int at[Pp::n];
#pragma unroll
    for (int r = 0; r < Pp::n; ++r) {
        const int t = Pp::cell(r);
        const int row = t / Wh, m = t - row * Wh;
        const int i = k + row / W, j = k + row % W;
        const int q = (i + j + k + p0 + colour) & 1;
        const int z = k + 2 * m + q;
        const int c = (i * S + j) * S + z;
        const T s = ((su[c - S * S] + su[c + S * S]) + (su[c - S] + su[c + S])) + (su[c - 1] + su[c + 1]);
        v[r] = (s - h2 * sf[((i - 1) * SF + (j - 1)) * SF + (z - 1)]) / T(6);
        at[r] = c;
    }
#pragma unroll
    for (int r = 0; r < Pp::n; ++r)
        if (Pp::live(r)) su[at[r]] = v[r];
}

template <class T, int S, int k, int kend>
__device__ __forceinline__ void lds_sweeps(T* su, const T* sf, T h2, int p0) {
    if constexpr (k <= kend) {
        lds_half_sweep<T, S, k>(su, sf, h2, (k - 1) & 1, p0);   // red (0) first
        __syncthreads();
        lds_sweeps<T, S, k + 1, kend>(su, sf, h2, p0);
    }
}

// v[S^3 region with origin o - R] = a[cell] (periodic wrap), into LDS
template <class T, int S>
__device__ __forceinline__ void load_region(T* dst, const T* __restrict__ a, int lg, int ox, int oy, int oz, int R) {
    using Pp = Passes<S * S * S>;
    const unsigned msk = (1u << lg) - 1;
    T v[Pp::n];
#pragma unroll
    for (int r = 0; r < Pp::n; ++r) {
        const int t = Pp::cell(r);
        const int i = t / (S * S), j = (t / S) % S, m = t % S;
        v[r] = a[sidx(lg, (unsigned)(ox - R + i) & msk, (unsigned)(oy - R + j) & msk, (unsigned)(oz - R + m) & msk)];
    }
#pragma unroll
    for (int r = 0; r < Pp::n; ++r)
        if (Pp::live(r)) dst[(int)threadIdx.x + r * kFusedThreads] = v[r];
}

// pre leg on level (edge 2^lg): u, f are the level's arrays as the parent's restriction left
// them; uo, fo receive the smoothed u and the FAS right-hand side of this tile; pu, pf, uold the
// restricted u, the restricted residual and its copy for the coarse level (edge 2^(lg-1))
template <class T, int NU>
__global__ void __launch_bounds__(kFusedThreads)
k_level_pre(const T* __restrict__ u, const T* __restrict__ f, T* __restrict__ uo, T* __restrict__ fo,
            T* __restrict__ pu, T* __restrict__ pf, T* __restrict__ uold, int lg, T h2) {
    constexpr int R = 2 * NU + 1;      // u halo: 2 nu1 half-sweeps + the residual stencil
    constexpr int S = kTile + 2 * R, SF = S - 2;
    __shared__ T su[S * S * S];
    __shared__ T sf[SF * SF * SF];
    const int lt = lg - 3;
    const unsigned b = blockIdx.x;
    const int ox = (int)(b >> (2 * lt)) * kTile, oy = (int)((b >> lt) & ((1u << lt) - 1)) * kTile,
              oz = (int)(b & ((1u << lt) - 1)) * kTile;
    load_region<T, S>(su, u, lg, ox, oy, oz, R);
    load_region<T, SF>(sf, f, lg, ox, oy, oz, R - 1);
    __syncthreads();
    // FAS right-hand side on the f region: f += L u (u here is the restricted fine u)
    {
        using Pp = Passes<SF * SF * SF>;
        T v[Pp::n];
#pragma unroll
        for (int r = 0; r < Pp::n; ++r) {
            const int t = Pp::cell(r);
            const int i = t / (SF * SF), j = (t / SF) % SF, m = t % SF;
            const int c = ((i + 1) * S + (j + 1)) * S + (m + 1);
            const T s = ((su[c - S * S] + su[c + S * S]) + (su[c - S] + su[c + S])) + (su[c - 1] + su[c + 1]);
            v[r] = sf[t] + (s - T(6) * su[c]) / h2;
        }
#pragma unroll
        for (int r = 0; r < Pp::n; ++r)
            if (Pp::live(r)) sf[(int)threadIdx.x + r * kFusedThreads] = v[r];
    }
    __syncthreads();
    lds_sweeps<T, S, 1, 2 * NU>(su, sf, h2, R & 1);
    // residual and restriction of the tile's 4^3 coarse cells: each thread one child, the 8
    // children of a coarse cell in 8 neighbouring lanes, summed in the order (a, b, e)
    {
        const int t = threadIdx.x, ch = t & 7, cc = t >> 3;
        const int X = cc >> 4, Y = (cc >> 2) & 3, Z = cc & 3;
        const int x = 2 * X + (ch >> 2), y = 2 * Y + ((ch >> 1) & 1), z = 2 * Z + (ch & 1);
        const int c = ((x + R) * S + (y + R)) * S + (z + R);
        const T ui = su[c];
        const T fi = sf[((x + R - 1) * SF + (y + R - 1)) * SF + (z + R - 1)];
        const T s = ((su[c - S * S] + su[c + S * S]) + (su[c - S] + su[c + S])) + (su[c - 1] + su[c + 1]);
        const T lap = (s - T(6) * ui) / h2;
        const T r = fi - lap;
        const int lane0 = (int)(threadIdx.x & 63) & ~7;
        T sr = T(0), sum_u = T(0);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            sr = sr + __shfl(r, lane0 + q, 64);
            sum_u = sum_u + __shfl(ui, lane0 + q, 64);
        }
        if (ch == 0) {
            const unsigned Xg = (unsigned)(ox / 2 + X), Yg = (unsigned)(oy / 2 + Y), Zg = (unsigned)(oz / 2 + Z);
            const int lc = lg - 1;
            const T uc = sum_u * T(0.125);
            const unsigned P = sidx(lc, Xg, Yg, Zg);
            pu[P] = uc;
            pf[P] = sr * T(0.125);
            uold[(((Xg << lc) | Yg) << lc) | Zg] = uc;
        }
        // the tile itself: smoothed u and the FAS right-hand side
        const unsigned g = sidx(lg, (unsigned)(ox + x), (unsigned)(oy + y), (unsigned)(oz + z));
        uo[g] = ui;
        fo[g] = fi;
    }
}

// post leg: u = ui + (uc[parent] - uold[parent]) over the tile and a halo of 2 nu2 cells, then
// nu2 red-black sweeps; the tile is written to uout.  fi is the FAS right-hand side of the level.
template <class T, int NU>
__global__ void __launch_bounds__(kFusedThreads)
k_level_post(const T* __restrict__ ui, const T* __restrict__ fi, const T* __restrict__ uc,
             const T* __restrict__ uold, T* __restrict__ uout, int lg, T h2) {
    constexpr int R = 2 * NU;
    constexpr int S = kTile + 2 * R, SF = S - 2;
    __shared__ T su[S * S * S];
    __shared__ T sf[SF * SF * SF];
    const int lt = lg - 3, lc = lg - 1;
    const unsigned b = blockIdx.x, msk = (1u << lg) - 1;
    const int ox = (int)(b >> (2 * lt)) * kTile, oy = (int)((b >> lt) & ((1u << lt) - 1)) * kTile,
              oz = (int)(b & ((1u << lt) - 1)) * kTile;
    {
        using Pp = Passes<S * S * S>;
        T v[Pp::n];
#pragma unroll
        for (int r = 0; r < Pp::n; ++r) {
            const int t = Pp::cell(r);
            const int i = t / (S * S), j = (t / S) % S, m = t % S;
            const unsigned x = (unsigned)(ox - R + i) & msk, y = (unsigned)(oy - R + j) & msk,
                           z = (unsigned)(oz - R + m) & msk;
            const unsigned X = x >> 1, Y = y >> 1, Z = z >> 1;
            v[r] = ui[sidx(lg, x, y, z)] + (uc[sidx(lc, X, Y, Z)] - uold[(((X << lc) | Y) << lc) | Z]);
        }
#pragma unroll
        for (int r = 0; r < Pp::n; ++r)
            if (Pp::live(r)) su[(int)threadIdx.x + r * kFusedThreads] = v[r];
    }
    load_region<T, SF>(sf, fi, lg, ox, oy, oz, R - 1);
    __syncthreads();
    lds_sweeps<T, S, 1, 2 * NU>(su, sf, h2, R & 1);
    {
        const int t = threadIdx.x;
        const int x = t >> 6, y = (t >> 3) & 7, z = t & 7;
        uout[sidx(lg, (unsigned)(ox + x), (unsigned)(oy + y), (unsigned)(oz + z))] = su[((x + R) * S + (y + R)) * S + (z + R)];
    }
}

// ----------------------------------------------------------------------------------------------
// One-step transfer kernels for periodic colour-split power-of-two cubes (the larger levels of a
// power-of-two base), with the same arithmetic as the generic ones and coalesced accesses: the
// lanes of a wave take consecutive coarse cells Z of a row, whose fine cells sit at consecutive
// positions of the fine half-rows.
// ----------------------------------------------------------------------------------------------

// Block order of the power-of-two kernels on large levels (the 16-byte half-sweeps and the
// residual-restriction).  Consecutive blocks go to the 8 XCDs in turn, so the rows at the edges
// of a block's run were fetched again into another XCD's L2 by the neighbouring blocks (counters
// at 256^3: 1.09x the compulsory bytes for the half-sweep, 1.22x for the residual-restriction).
// Within each group of 32 blocks the order is permuted so that 4 consecutive runs share an XCD
// (hardware block b takes run 4 (b mod 8) + (b div 8) mod 4); the interleave across XCDs stays
// fine-grained.  Applied only where an x plane spans a multiple of 32 blocks, so that
// x-neighbouring planes keep sharing an XCD (at 128^3 a half-sweep plane is 8 blocks, and the
// permutation measured slower there).  Measured at 256^3: half-sweep counters 1.02x, FP32
// 16.7 -> 16.4 us; residual-restriction fetch -15%, FP32 26.0 -> 24.8 us.
__device__ __forceinline__ unsigned xcd_quads(unsigned b, unsigned grid, unsigned blocks_per_plane) {
    if (grid % 32 != 0 || blocks_per_plane % 32 != 0) return b;
    return (b & ~31u) | (((b & 7u) << 2) | ((b >> 3) & 3u));
}

// steps 3-5, one thread per coarse cell (cell_resid_restrict_p2)
template <class T>
__global__ void __launch_bounds__(256)
k_resid_restrict_p2(const T* __restrict__ u, const T* __restrict__ f, int lg, T h2, T* __restrict__ pu,
                    T* __restrict__ pf, T* __restrict__ uold) {
    const int lc = lg - 1;
    const unsigned t = xcd_quads(blockIdx.x, gridDim.x, (1u << (2 * lc)) / blockDim.x) * blockDim.x + threadIdx.x;
    if (t >= 1u << (3 * lc)) return;
    cell_resid_restrict_p2<T>(u, f, lg, h2, pu, pf, uold, t);
}

// step 8 on the black cells: the black cell (row, j) of a fine row lies in the parent (X, Y, j)
template <class T>
__global__ void __launch_bounds__(256)
k_prolong_black_p2(T* __restrict__ u, int lg, const T* __restrict__ pu, const T* __restrict__ uold) {
    const int lc = lg - 1;
    const unsigned nzh = 1u << lc, m = (1u << lg) - 1;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 1u << (3 * lg - 1)) return;
    const unsigned row = t >> lc, j = t & (nzh - 1);
    const unsigned x = row >> lg, y = row & m;
    const unsigned X = x >> 1, Y = y >> 1;
    const unsigned i = (row << lg) + nzh + j;
    u[i] = u[i] + (pu[sidx(lc, X, Y, j)] - uold[(((X << lc) | Y) << lc) | j]);
}

// step 6 on a whole periodic coarse level (edge 2^lg): f += L u for the cell t (natural order)
template <class T>
__global__ void __launch_bounds__(256)
k_fas_rhs_p2(const T* __restrict__ pu, T* __restrict__ pf, int lg, T H2) {
    const unsigned m = (1u << lg) - 1;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 1u << (3 * lg)) return;
    const unsigned x = t >> (2 * lg), y = (t >> lg) & m, z = t & m;
    const unsigned i = sidx(lg, x, y, z);
    const T s = ((pu[sidx(lg, (x - 1) & m, y, z)] + pu[sidx(lg, (x + 1) & m, y, z)]) +
                 (pu[sidx(lg, x, (y - 1) & m, z)] + pu[sidx(lg, x, (y + 1) & m, z)])) +
                (pu[sidx(lg, x, y, (z - 1) & m)] + pu[sidx(lg, x, y, (z + 1) & m)]);
    pf[i] = pf[i] + (s - T(6) * pu[i]) / H2;
}

template <class T>
void launch_resid_restrict_p2(const T* u, const T* f, int n, double h, T* pu, T* pf, T* uold, hipStream_t st) {
    const int lg = __builtin_ctz((unsigned)n);
    const unsigned cells = 1u << (3 * (lg - 1));
    k_resid_restrict_p2<T><<<(cells + 255) / 256, 256, 0, st>>>(u, f, lg, (T)(h * h), pu, pf, uold);
}

// step 8 on the black cells, W at a time with 16-byte accesses (run_prolong_black_vec)
template <class T>
__global__ void __launch_bounds__(256)
k_prolong_black_vec(T* __restrict__ u, int lg, const T* __restrict__ pu, const T* __restrict__ uold) {
    constexpr int W = Vec16<T>::W;
    const unsigned ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch < (1u << (3 * lg - 1 - __builtin_ctz(W)))) run_prolong_black_vec<T>(u, lg, pu, uold, ch);
}

template <class T>
void launch_prolong_black_p2(T* u, int n, const T* pu, const T* uold, hipStream_t st) {
    constexpr int W = Vec16<T>::W;
    const int lg = __builtin_ctz((unsigned)n);
    const unsigned cells = 1u << (3 * lg - 1);
    if ((1u << (lg - 1)) % W == 0) {   // half-rows hold whole runs
        const unsigned runs = cells / W;
        k_prolong_black_vec<T><<<(runs + 255) / 256, 256, 0, st>>>(u, lg, pu, uold);
    } else {
        k_prolong_black_p2<T><<<(cells + 255) / 256, 256, 0, st>>>(u, lg, pu, uold);
    }
}

template <class T>
void launch_fas_rhs_p2(const T* pu, T* pf, int n, double H, hipStream_t st) {
    const int lg = __builtin_ctz((unsigned)n);
    const unsigned cells = 1u << (3 * lg);
    k_fas_rhs_p2<T><<<(cells + 255) / 256, 256, 0, st>>>(pu, pf, lg, (T)(H * H));
}

// ----------------------------------------------------------------------------------------------
// Red-black half-sweep on a periodic colour-split power-of-two level with 16-byte accesses: a
// thread takes W = 16 / sizeof(T) consecutive cells j0 .. j0 + W - 1 of its colour in one
// half-row (4 FP32 or 2 FP64 cells) and reads each neighbour run, f and the other colour's entries
// of its own row as one vector; the one z-neighbour outside that run (entry j0 - 1 or j0 + W of
// the other half, by the row's parity) is a scalar load.  Each cell is updated with the
// expression of cell_rbgs_split, so the bits are the same.
// ----------------------------------------------------------------------------------------------
template <class T, int CH>
__global__ void __launch_bounds__(256)
k_rbgs_vec(T* __restrict__ u, const T* __restrict__ f, int lgx, int lgy, int lgz, T h2, int colour) {
    constexpr int W = Vec16<T>::W;
    const unsigned lzh = (unsigned)lgz - 1;
    const unsigned chunks = 1u << (lgx + lgy + lzh - __builtin_ctz(W));   // W-cell runs of one colour
    const unsigned bl = xcd_quads(blockIdx.x, gridDim.x, (1u << (lgy + lzh - __builtin_ctz(W))) / (CH * blockDim.x));
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const unsigned ch = (bl * CH + c) * blockDim.x + threadIdx.x;
        if (ch >= chunks) break;
        run_rbgs_vec<T>(u, f, lgx, lgy, lgz, h2, colour, ch);
    }
}

// The first red half-sweep after the coarse-grid correction (step 8 then step 9), in one pass:
// the correction u += pu[parent] - uold[parent] of the black cells is only ever read by this
// half-sweep (the black half-sweep after it rewrites every black cell without reading it), so it
// is applied here to each black value as it is read, and never stored.  A black cell (row, j) of
// the fine level lies in the parent (x >> 1, y >> 1, j); the parents of a run of W black cells are
// W consecutive Z of one coarse row: a vector of uold (natural order) and two half-vectors of pu
// (colour-split order, even and odd Z in the two halves).  Same arithmetic as k_prolong_black_p2
// followed by k_rbgs_vec, so the same bits.
// d[k] = pu - uold for the parents (X, Y, j0 + k) of a run of W black cells
template <class T>
__device__ __forceinline__ void corr_delta(const T* __restrict__ pu, const T* __restrict__ uold, int lc, unsigned X,
                                           unsigned Y, unsigned j0, T* d) {
    constexpr int W = Vec16<T>::W;
    const unsigned nch = (1u << lc) >> 1;
    const unsigned rb = ((X << lc) | Y) << lc;
    const unsigned he = ((X + Y) & 1u) * nch, ho = nch - he;   // halves holding even / odd Z
    const typename Vec16<T>::type o = *(const typename Vec16<T>::type*)(uold + rb + j0);
    if constexpr (W == 4) {
        const float2 pe = *(const float2*)(pu + rb + he + (j0 >> 1)), po = *(const float2*)(pu + rb + ho + (j0 >> 1));
        d[0] = pe.x - o.x;
        d[1] = po.x - o.y;
        d[2] = pe.y - o.z;
        d[3] = po.y - o.w;
    } else {
        d[0] = pu[rb + he + (j0 >> 1)] - o.x;
        d[1] = pu[rb + ho + (j0 >> 1)] - o.y;
    }
}

template <class T>
__global__ void __launch_bounds__(256)
k_rbgs_vec_corr(T* __restrict__ u, const T* __restrict__ f, int lgx, int lgy, int lgz, T h2,
                const T* __restrict__ pu, const T* __restrict__ uold) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    const unsigned lzh = (unsigned)lgz - 1, nzh = 1u << lzh, mx = (1u << lgx) - 1, my = (1u << lgy) - 1;
    const int lc = lgz - 1;                        // the coarse level is a cube of edge 2^(lgz - 1)
    const unsigned chunks = 1u << (lgx + lgy + lzh - __builtin_ctz(W));
    const unsigned bl = xcd_quads(blockIdx.x, gridDim.x, (1u << (lgy + lzh - __builtin_ctz(W))) / blockDim.x);
    const unsigned ch = bl * blockDim.x + threadIdx.x;
    if (ch >= chunks) return;
    const unsigned t = ch * W, row = t >> lzh, j0 = t & (nzh - 1);
    const unsigned x = row >> lgy, y = row & my;
    const unsigned q = (x + y) & 1u;              // z parity of red cells in the row
    const unsigned r0 = row << lgz;
    const unsigned xm = (x - 1) & mx, xp = (x + 1) & mx, ym = (y - 1) & my, yp = (y + 1) & my;
    // the black runs read are those of rows x-1, x+1, y-1, y+1 and the own row; their parents lie in
    // the own parent row (X, Y) and in one more row along x (for x-1 if x is even, else x+1) and
    // one along y, so three correction runs cover all five
    const unsigned X = x >> 1, Y = y >> 1;
    T dO[W], dX[W], dY[W];
    corr_delta<T>(pu, uold, lc, X, Y, j0, dO);
    corr_delta<T>(pu, uold, lc, ((x & 1u) ? xp : xm) >> 1, Y, j0, dX);
    corr_delta<T>(pu, uold, lc, X, ((y & 1u) ? yp : ym) >> 1, j0, dY);
    auto run = [&](unsigned xr, unsigned yr, const T* d, T* c) {
        const V v = *(const V*)(u + (((xr << lgy) | yr) << lgz) + nzh + j0);
#pragma unroll
        for (int k = 0; k < W; ++k) c[k] = lane<T>(v, k) + d[k];
    };
    T XM[W], XP[W], YM[W], YP[W], C[W];
    run(xm, y, (x & 1u) ? dO : dX, XM);
    run(xp, y, (x & 1u) ? dX : dO, XP);
    run(x, ym, (y & 1u) ? dO : dY, YM);
    run(x, yp, (y & 1u) ? dY : dO, YP);
    run(x, y, dO, C);
    // the one black entry of the own row outside the run (j0 - 1 or j0 + W, by parity), corrected
    const unsigned je = q ? ((j0 + W) & (nzh - 1)) : ((j0 - 1) & (nzh - 1));
    T edge;
    {
        const unsigned ncz = 1u << lc, rb = ((X << lc) | Y) << lc;
        edge = u[r0 + nzh + je] + (pu[rb + ((X + Y + je) & 1u) * (ncz >> 1) + (je >> 1)] - uold[rb + je]);
    }
    const V F = *(const V*)(f + r0 + j0);
    T out[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const T zm = q ? C[k] : (k == 0 ? edge : C[k - 1]);
        const T zp = q ? (k == W - 1 ? edge : C[k + 1]) : C[k];
        const T s = ((XM[k] + XP[k]) + (YM[k] + YP[k])) + (zm + zp);
        out[k] = (s - h2 * lane<T>(F, k)) / T(6);
    }
    V o;
    if constexpr (W == 4) o = V{out[0], out[1], out[2], out[3]};
    else o = V{out[0], out[1]};
    *(V*)(u + r0 + j0) = o;
}

template <class T>
void launch_rbgs_vec_corr(T* u, const T* f, const Lay& L, double h, const T* pu, const T* uold, hipStream_t st) {
    constexpr int W = Vec16<T>::W;
    const unsigned chunks = (unsigned)(L.d.cells() / 2 / W);
    k_rbgs_vec_corr<T><<<(chunks + 255) / 256, 256, 0, st>>>(u, f, L.lgx, L.lgy, L.lgz, (T)(h * h), pu, uold);
}

// Step 6 on a whole periodic colour-split power-of-two level with 16-byte accesses (run_fas_vec:
// a thread takes the runs j0 .. j0 + W - 1 of both colours of one row).
template <class T>
__global__ void __launch_bounds__(256)
k_fas_vec(const T* __restrict__ pu, T* __restrict__ pf, int lg, T H2) {
    constexpr int W = Vec16<T>::W;
    const unsigned chunks = 1u << (3 * lg - 1 - __builtin_ctz(W));   // runs per colour
    const unsigned ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch < chunks) run_fas_vec<T>(pu, pf, lg, H2, ch);
}

template <class T>
void launch_fas_vec(const T* pu, T* pf, int n, double H, hipStream_t st) {
    constexpr int W = Vec16<T>::W;
    const int lg = __builtin_ctz((unsigned)n);
    const unsigned chunks = (unsigned)((size_t)n * n * n / 2 / W);
    k_fas_vec<T><<<(chunks + 255) / 256, 256, 0, st>>>(pu, pf, lg, (T)(H * H));
}

bool rbgs_vec_ok(const Lay& L, size_t elem) {
    const unsigned W = 16u / (unsigned)elem;
    return L.pow2 && L.split && L.lgz >= 1 && ((1u << (L.lgz - 1)) % W) == 0;
}

template <class T>
void launch_rbgs_vec(T* u, const T* f, const Lay& L, double h, int colour, hipStream_t st, hipEvent_t ev0,
                     hipEvent_t ev1) {
    constexpr int W = Vec16<T>::W;
    const unsigned chunks = (unsigned)(L.d.cells() / 2 / W);
    const T h2 = (T)(h * h);
    // measured: 1 run per thread is best for FP32 at 128^3 and 256^3 and for FP64 at 128^3; FP64
    // at 256^3 and above is 5% faster with 2
    // stamped by the events when they are given (kernel timing), else a plain launch (the form
    // captured into graphs)
    if (sizeof(T) == 8 && chunks >= (1u << 22)) {
        if (ev0)
            hipExtLaunchKernelGGL(k_rbgs_vec<T, 2>, dim3((chunks + 511) / 512), dim3(256), 0, st, ev0, ev1, 0, u, f,
                                  L.lgx, L.lgy, L.lgz, h2, colour);
        else
            k_rbgs_vec<T, 2><<<(chunks + 511) / 512, 256, 0, st>>>(u, f, L.lgx, L.lgy, L.lgz, h2, colour);
    } else {
        if (ev0)
            hipExtLaunchKernelGGL(k_rbgs_vec<T, 1>, dim3((chunks + 255) / 256), dim3(256), 0, st, ev0, ev1, 0, u, f,
                                  L.lgx, L.lgy, L.lgz, h2, colour);
        else
            k_rbgs_vec<T, 1><<<(chunks + 255) / 256, 256, 0, st>>>(u, f, L.lgx, L.lgy, L.lgz, h2, colour);
    }
}

bool level_fusable(int n, int nu1, int nu2) {
    return (n == 16 || n == 32 || n == 64) && nu1 >= 1 && nu1 <= 2 && nu2 >= 1 && nu2 <= 2;
}

template <class T>
void launch_level_pre(const T* u, const T* f, T* uo, T* fo, T* pu, T* pf, T* uold, int n, double h, int nu1,
                      hipStream_t st) {
    const int lg = __builtin_ctz((unsigned)n);
    const unsigned tiles = 1u << (3 * (lg - 3));
    const T h2 = (T)(h * h);
    if (nu1 == 1) k_level_pre<T, 1><<<tiles, kFusedThreads, 0, st>>>(u, f, uo, fo, pu, pf, uold, lg, h2);
    else k_level_pre<T, 2><<<tiles, kFusedThreads, 0, st>>>(u, f, uo, fo, pu, pf, uold, lg, h2);
}

template <class T>
void launch_level_post(const T* ui, const T* fi, const T* uc, const T* uold, T* uout, int n, double h, int nu2,
                       hipStream_t st) {
    const int lg = __builtin_ctz((unsigned)n);
    const unsigned tiles = 1u << (3 * (lg - 3));
    const T h2 = (T)(h * h);
    if (nu2 == 1) k_level_post<T, 1><<<tiles, kFusedThreads, 0, st>>>(ui, fi, uc, uold, uout, lg, h2);
    else k_level_post<T, 2><<<tiles, kFusedThreads, 0, st>>>(ui, fi, uc, uold, uout, lg, h2);
}

#define MG_INST(T)                                                                                      \
    template void launch_resid_restrict_p2<T>(const T*, const T*, int, double, T*, T*, T*, hipStream_t);      \
    template void launch_prolong_black_p2<T>(T*, int, const T*, const T*, hipStream_t);                       \
    template void launch_fas_rhs_p2<T>(const T*, T*, int, double, hipStream_t);                               \
    template void launch_rbgs_vec<T>(T*, const T*, const Lay&, double, int, hipStream_t, hipEvent_t, hipEvent_t); \
    template void launch_rbgs_vec_corr<T>(T*, const T*, const Lay&, double, const T*, const T*, hipStream_t);     \
    template void launch_fas_vec<T>(const T*, T*, int, double, hipStream_t);                                  \
    template void launch_level_pre<T>(const T*, const T*, T*, T*, T*, T*, T*, int, double, int, hipStream_t); \
    template void launch_level_post<T>(const T*, const T*, const T*, const T*, T*, int, double, int, hipStream_t);
MG_INST(float)
MG_INST(double)
#undef MG_INST

}  // namespace mgic
