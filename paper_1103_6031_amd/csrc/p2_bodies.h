// Per-thread bodies for colour-split power-of-two periodic levels (Section 3.2), shared by the
// solo kernels (k_levels.hip) and the batched ones (k_multigrid.hip): the red-black half-sweep
// and the FAS right-hand side on 16-byte runs, the black-cell prolongation on 16-byte runs, and
// the residual + restriction of one coarse cell.
#pragma once

#include <hip/hip_runtime.h>

namespace mgic {

template <class T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int W = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int W = 2; };

template <class T>
__device__ __forceinline__ T lane(const typename Vec16<T>::type& v, int k) {
    if constexpr (Vec16<T>::W == 4) return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
    else return k == 0 ? v.x : v.y;
}

// Half-sweep of `colour` on the run ch (W consecutive cells of the colour in one half-row) of a
// periodic colour-split cube of edges 2^lgx, 2^lgy, 2^lgz whose half-rows hold a multiple of W
// cells.  Each neighbour run (x +- 1, y +- 1 rows), f and the other colour's entries of the own
// row are read as one 16-byte vector; the one z-neighbour outside the run is a scalar load.  Each
// cell has the operations of the one-cell-per-thread half-sweep, so the bits are the same.
template <class T>
__device__ __forceinline__ void run_rbgs_vec(T* __restrict__ u, const T* __restrict__ f, int lgx, int lgy, int lgz,
                                             T h2, int colour, unsigned ch) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    const unsigned lzh = (unsigned)lgz - 1, nzh = 1u << lzh, mx = (1u << lgx) - 1, my = (1u << lgy) - 1;
    const unsigned own = colour ? nzh : 0u, oth = colour ? 0u : nzh;
    const unsigned t = ch * W;                 // first cell of the run in the colour's order
    const unsigned row = t >> lzh, j0 = t & (nzh - 1);
    const unsigned x = row >> lgy, y = row & my;
    const unsigned q = (x + y + (unsigned)colour) & 1u;   // z parity of this colour in the row
    const unsigned r0 = row << lgz;
    const unsigned rxm = ((((x - 1) & mx) << lgy) | y) << lgz, rxp = ((((x + 1) & mx) << lgy) | y) << lgz;
    const unsigned rym = ((x << lgy) | ((y - 1) & my)) << lgz, ryp = ((x << lgy) | ((y + 1) & my)) << lgz;
    const V XM = *(const V*)(u + rxm + oth + j0), XP = *(const V*)(u + rxp + oth + j0);
    const V YM = *(const V*)(u + rym + oth + j0), YP = *(const V*)(u + ryp + oth + j0);
    const V C = *(const V*)(u + r0 + oth + j0);    // the other colour's entries j0 .. j0 + W - 1
    const V F = *(const V*)(f + r0 + own + j0);
    // cell j = j0 + k sits at z = 2j + q; its z-neighbours are the other colour's entries
    // j - 1 + q and j + q: for q = 0 these are C[k - 1] (entry j0 - 1 for k = 0) and C[k],
    // for q = 1 C[k] and C[k + 1] (entry j0 + W for k = W - 1)
    const T edge = u[r0 + oth + (q ? ((j0 + W) & (nzh - 1)) : ((j0 - 1) & (nzh - 1)))];
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
}

// position of (x, y, z) in a colour-split power-of-two cube of edge 2^lg
__device__ __forceinline__ unsigned sidx(int lg, unsigned x, unsigned y, unsigned z) {
    return ((((x << lg) | y) << lg) + (((x + y + z) & 1u) << (lg - 1))) + (z >> 1);
}

// steps 3-5 for the coarse cell t = (X, Y, Z) (natural order) of a periodic colour-split
// power-of-two cube of fine edge 2^lg: the 8 children's residuals and values summed in the order
// (a, b, e), the order of the generic residual-restriction, so the bits are the same.  The
// children and their neighbours span the fine rows (2X + a, 2Y + b) at z = 2Z - 1 .. 2Z + 2, and
// the rows one step outside in x and in y at z = 2Z, 2Z + 1; in a row whose even-z cells are
// colour p, z = 2Z and 2Z + 2 are entries Z and Z + 1 of half p, z = 2Z - 1 and 2Z + 1 entries
// Z - 1 and Z of the other half.
template <class T>
__device__ __forceinline__ void cell_resid_restrict_p2(const T* __restrict__ u, const T* __restrict__ f, int lg, T h2,
                                                       T* __restrict__ pu, T* __restrict__ pf, T* __restrict__ uold,
                                                       unsigned t) {
    const int lc = lg - 1;
    const unsigned nc = 1u << lc, mc = nc - 1, m = (1u << lg) - 1, nzh = nc;
    const unsigned X = t >> (2 * lc), Y = (t >> lc) & mc, Z = t & mc;
    const unsigned x0 = 2 * X, y0 = 2 * Y;
    const unsigned Zm = (Z - 1) & mc, Zp = (Z + 1) & mc;
    auto rowb = [&](unsigned x, unsigned y) { return (((x & m) << lg) | (y & m)) << lg; };
    auto half = [&](unsigned x, unsigned y, unsigned zpar) {   // offset of the half holding parity zpar
        return ((x + y + zpar) & 1u) * nzh;
    };
    // central rows (a, b): values at z0 - 1, z0, z0 + 1, z0 + 2 and f at z0, z0 + 1
    T cm[2][2], c0[2][2], c1[2][2], c2[2][2], f0[2][2], f1[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const unsigned x = x0 + a, y = y0 + b, rb = rowb(x, y);
            const unsigned he = half(x, y, 0), ho = half(x, y, 1);
            cm[a][b] = u[rb + ho + Zm];
            c0[a][b] = u[rb + he + Z];
            c1[a][b] = u[rb + ho + Z];
            c2[a][b] = u[rb + he + Zp];
            f0[a][b] = f[rb + he + Z];
            f1[a][b] = f[rb + ho + Z];
        }
    // face rows: x0 - 1 and x0 + 2 (for b = 0, 1), y0 - 1 and y0 + 2 (for a = 0, 1), at z0, z0 + 1
    T xf[2][2][2], yf[2][2][2];   // [side][b or a][e]
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            {
                const unsigned x = sd ? x0 + 2 : x0 - 1, y = y0 + k, rb = rowb(x, y);
                xf[sd][k][0] = u[rb + half(x, y, 0) + Z];
                xf[sd][k][1] = u[rb + half(x, y, 1) + Z];
            }
            {
                const unsigned x = x0 + k, y = sd ? y0 + 2 : y0 - 1, rb = rowb(x, y);
                yf[sd][k][0] = u[rb + half(x, y, 0) + Z];
                yf[sd][k][1] = u[rb + half(x, y, 1) + Z];
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
    const unsigned P = sidx(lc, X, Y, Z);
    pu[P] = uc;
    pf[P] = sr * T(0.125);
    uold[t] = uc;
}

// Step 6 on a whole periodic colour-split power-of-two level (edge 2^lg) for the run ch: the
// cells j0 .. j0 + W - 1 of both colours of one row (the red run's neighbours are the black runs
// of the 4 neighbour rows and the black run of its own row, and the other way round) take
// pf += (nsum(pu) - 6 pu) / H2 with the arithmetic of the one-cell-per-thread kernel.
template <class T>
__device__ __forceinline__ void run_fas_vec(const T* __restrict__ pu, T* __restrict__ pf, int lg, T H2, unsigned ch) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    const unsigned lzh = (unsigned)lg - 1, nzh = 1u << lzh, m = (1u << lg) - 1;
    const unsigned t = ch * W, row = t >> lzh, j0 = t & (nzh - 1);
    const unsigned x = row >> lg, y = row & m;
    const unsigned r0 = row << lg;
    const unsigned rxm = ((((x - 1) & m) << lg) | y) << lg, rxp = ((((x + 1) & m) << lg) | y) << lg;
    const unsigned rym = ((x << lg) | ((y - 1) & m)) << lg, ryp = ((x << lg) | ((y + 1) & m)) << lg;
    const V own[2] = {*(const V*)(pu + r0 + j0), *(const V*)(pu + r0 + nzh + j0)};   // red, black runs
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const unsigned oth = c ? 0u : nzh, mine = c ? nzh : 0u;
        const unsigned q = (x + y + (unsigned)c) & 1u;   // z parity of colour c in the row
        const V XM = *(const V*)(pu + rxm + oth + j0), XP = *(const V*)(pu + rxp + oth + j0);
        const V YM = *(const V*)(pu + rym + oth + j0), YP = *(const V*)(pu + ryp + oth + j0);
        const V& C = own[1 - c];
        const T edge = pu[r0 + oth + (q ? ((j0 + W) & (nzh - 1)) : ((j0 - 1) & (nzh - 1)))];
        const V Fv = *(const V*)(pf + r0 + mine + j0);
        T out[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const T zm = q ? lane<T>(C, k) : (k == 0 ? edge : lane<T>(C, k - 1));
            const T zp = q ? (k == W - 1 ? edge : lane<T>(C, k + 1)) : lane<T>(C, k);
            const T s = ((lane<T>(XM, k) + lane<T>(XP, k)) + (lane<T>(YM, k) + lane<T>(YP, k))) + (zm + zp);
            out[k] = lane<T>(Fv, k) + (s - T(6) * lane<T>(own[c], k)) / H2;
        }
        V o;
        if constexpr (W == 4) o = V{out[0], out[1], out[2], out[3]};
        else o = V{out[0], out[1]};
        *(V*)(pf + r0 + mine + j0) = o;
    }
}

// Step 8 on the black cells of a periodic colour-split power-of-two level (edge 2^lg, half-rows a
// multiple of W) for the run ch: black cells j0 .. j0 + W - 1 of one fine row.  The black cell j
// of fine row (x, y) lies in the parent cell (x / 2, y / 2, j), so the run's parents are W
// consecutive cells of one coarse row: consecutive in uold (natural order), alternating between
// the two colour halves of the colour-split parent (even z in the half of parity x/2 + y/2).
// Each cell takes u += pu - uold as the one-cell-per-thread kernel does.
template <class T>
__device__ __forceinline__ void run_prolong_black_vec(T* __restrict__ u, int lg, const T* __restrict__ pu,
                                                      const T* __restrict__ uold, unsigned ch) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    const unsigned lzh = (unsigned)lg - 1, nzh = 1u << lzh, m = (1u << lg) - 1;
    const int lc = lg - 1;
    const unsigned t = ch * W, row = t >> lzh, j0 = t & (nzh - 1);
    const unsigned x = row >> lg, y = row & m, X = x >> 1, Y = y >> 1;
    const unsigned crow = ((X << lc) | Y) << lc;
    const unsigned ev = ((X + Y) & 1u) << (lc - 1), od = (((X + Y) & 1u) ^ 1u) << (lc - 1);
    T* const ur = u + (row << lg) + nzh + j0;
    const V U = *(const V*)ur;
    const V O = *(const V*)(uold + crow + j0);
    T pe[W / 2], po[W / 2];   // parents at z = j0 + 2i and j0 + 2i + 1
    if constexpr (W == 4) {
        const float2 a = *(const float2*)(pu + crow + ev + (j0 >> 1));
        const float2 b = *(const float2*)(pu + crow + od + (j0 >> 1));
        pe[0] = a.x; pe[1] = a.y; po[0] = b.x; po[1] = b.y;
    } else {
        pe[0] = pu[crow + ev + (j0 >> 1)];
        po[0] = pu[crow + od + (j0 >> 1)];
    }
    T out[W];
#pragma unroll
    for (int k = 0; k < W; ++k) out[k] = lane<T>(U, k) + ((k & 1 ? po[k >> 1] : pe[k >> 1]) - lane<T>(O, k));
    V o;
    if constexpr (W == 4) o = V{out[0], out[1], out[2], out[3]};
    else o = V{out[0], out[1]};
    *(V*)ur = o;
}

}  // namespace mgic
