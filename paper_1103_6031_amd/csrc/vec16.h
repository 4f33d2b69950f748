// 16-byte runs on colour-split power-of-two periodic levels (Section 3.2 red-black half-sweep),
// shared by the solo kernels (k_levels.hip) and the batched ones (k_multigrid.hip).
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

}  // namespace mgic
