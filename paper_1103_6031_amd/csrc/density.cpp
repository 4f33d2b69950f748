// Host side of the multi-scale density (Hahn & Abel 2011, Sections 2.1-2.3 and 3.5.3): kernels
// per level, mode-preserving noise refinement and the nested convolutions, scheduled on the
// three-pass FFT of k_fft.hip and the grid kernels of k_density.hip.
//
// Levels: 0 is the periodic base (N^3); patch p has n_p cells per axis and the padded domain D'_p
// of 2 n_p cells per axis centred on it (the patch at [n_p/2, 3 n_p/2) of D'_p).  Per level the
// workspace holds the noise (N^3, or (2 n_p)^3 on D'_p) and the kernel grid, which is transformed
// in place into its (real) spectrum.  Convolutions are circular on the base or on D'_p.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "spec_internal.h"
#include "mgic.h"

namespace mgic {

namespace {

#define DN_HIP(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            return report_error(MG_EHIP, (std::string(#call) + ": " + hipGetErrorString(e_)).c_str()); \
        }                                                                                        \
    } while (0)

size_t cells3(const int* n) { return (size_t)n[0] * n[1] * n[2]; }

struct DensLevel {
    int n[3];        // own cells
    int off[3];      // in parent cells (patches)
    int D[3];        // noise / kernel grid: N (base) or 2 n (patch)
    double h;
    double* mu = nullptr;    // noise, D cells
    double* T = nullptr;     // kernel grid, then its spectrum, D cells
    SpecGrid G;              // transforms on D (periodic)
    SpecGrid R;              // the parent region under D' (n cells per axis, periodic) - patches
};

struct DensPlan {
    int nl = 0;
    std::vector<DensLevel> L;
    double* reg = nullptr;       // gathered parent region (max n^3)
    double2* csp = nullptr;      // its spectrum
    double* a = nullptr;         // convolution inputs / outputs on D' (max (2n)^3)
    double* b = nullptr;
    double* c = nullptr;
    double* zbase = nullptr;     // base noise with the first patch's cells zeroed (N^3)
    double* carry0 = nullptr;    // the base's coarse contribution (N^3)
    double* carryA = nullptr;    // coarse contributions on patches (max n^3), ping-pong
    double* carryB = nullptr;
    size_t bytes = 0;
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int dens_plan(const mg_hier* H, void* ws, DensPlan& P) {
    if (!H) return report_error(MG_EINVAL, "hierarchy is NULL");
    if (H->nlev < 1 || H->nlev > MG_MAX_LEVELS) return report_error(MG_EINVAL, "nlev out of range");
    const mg_level& b = H->lev[0];
    const int N = b.n[0];
    if (b.n[1] != N || b.n[2] != N) return report_error(MG_EINVAL, "base must be cubic");
    if (log2_exact(N) < 1 || N > 1024) return report_error(MG_EINVAL, "base must be a power of two in 2..1024");
    if (!(b.h > 0) || !std::isfinite(b.h)) return report_error(MG_EINVAL, "base spacing must be positive");
    P.nl = H->nlev;
    P.L.assign(P.nl, DensLevel());
    for (int l = 0; l < P.nl; ++l) {
        const mg_level& v = H->lev[l];
        DensLevel& D = P.L[l];
        D.h = v.h;
        for (int a = 0; a < 3; ++a) {
            D.n[a] = v.n[a];
            D.off[a] = l ? v.off[a] : 0;
            D.D[a] = l ? 2 * v.n[a] : N;
        }
        if (l == 0) continue;
        const DensLevel& Q = P.L[l - 1];
        if (std::fabs(v.h - 0.5 * Q.h) > 1e-12 * Q.h) return report_error(MG_EINVAL, "patch spacing must be half its parent's");
        for (int a = 0; a < 3; ++a) {
            const int n = v.n[a], o = v.off[a];
            if (n < 4 || log2_exact(n) < 0 || 2 * n > 1024)
                return report_error(MG_EINVAL, "patch sizes must be powers of two in 4..512");
            if (l == 1) {
                if (o < 0 || o + n / 2 > N || n / 2 > N - 2 || n > N)
                    return report_error(MG_EINVAL, "first patch not properly nested in the base");
            } else {
                if (o < 4 || o + n / 2 > Q.n[a] - 4) return report_error(MG_EINVAL, "patch not properly nested in its parent");
                if (o - n / 4 < 0 || o + 3 * n / 4 > Q.n[a])
                    return report_error(MG_EINVAL, "padded domain of a patch leaves its parent");
            }
        }
    }
    size_t off = 0;
    char* base = (char*)ws;
    auto take = [&](size_t bytes) -> void* {
        off = al256(off);
        void* p = base ? (void*)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    size_t w1 = 0, w2 = 0, maxn = 0, maxd = 0;
    for (int l = 0; l < P.nl; ++l) {
        DensLevel& D = P.L[l];
        int rc = spec_grid_init(D.D, 0, D.G);
        if (rc) return rc;
        spec_grid_carve(D.G, base, off);
        size_t a1, a2;
        spec_grid_work(D.G, a1, a2);
        w1 = std::max(w1, a1);
        w2 = std::max(w2, a2);
        D.mu = (double*)take(sizeof(double) * cells3(D.D));
        D.T = (double*)take(sizeof(double) * cells3(D.D));
        if (l) {
            rc = spec_grid_init(D.n, 0, D.R);
            if (rc) return rc;
            spec_grid_carve(D.R, base, off);
            spec_grid_work(D.R, a1, a2);
            w1 = std::max(w1, a1);
            w2 = std::max(w2, a2);
            maxn = std::max(maxn, cells3(D.n));
            maxd = std::max(maxd, cells3(D.D));
        }
    }
    double2* W1 = (double2*)take(sizeof(double2) * w1);
    double2* W2 = (double2*)take(sizeof(double2) * w2);
    double2* W3 = (double2*)take(sizeof(double2) * w2);
    for (DensLevel& D : P.L) {
        D.G.W1 = D.R.W1 = W1;
        D.G.W2 = D.R.W2 = W2;
        D.G.W3 = D.R.W3 = W3;
    }
    const size_t nb = cells3(P.L[0].D);
    P.zbase = (double*)take(sizeof(double) * nb);
    P.carry0 = (double*)take(sizeof(double) * nb);
    if (P.nl > 1) {
        P.reg = (double*)take(sizeof(double) * maxn);
        P.csp = (double2*)take(sizeof(double2) * maxn);
        P.a = (double*)take(sizeof(double) * maxd);
        P.b = (double*)take(sizeof(double) * maxd);
        P.c = (double*)take(sizeof(double) * maxd);
        P.carryA = (double*)take(sizeof(double) * maxn);
        P.carryB = (double*)take(sizeof(double) * maxn);
    }
    P.bytes = al256(off);
    return MG_OK;
}

// the parent's noise (or any parent array of the same layout) as seen from patch l: the box of
// parent cells starting at lo (in the parent's own cells)
DensBox parent_box(const DensPlan& P, int l, const int* lo) {
    DensBox B;
    const DensLevel& Q = P.L[l - 1];
    for (int a = 0; a < 3; ++a) {
        B.pd[a] = Q.D[a];
        B.po[a] = l == 1 ? 0 : Q.n[a] / 2;
        B.lo[a] = lo[a];
    }
    B.wrap = l == 1 ? Q.n[0] : 0;
    return B;
}

// a parent array of the parent's own cells (no padding: the base, or a patch's n^3 array)
DensBox parent_plain_box(const DensPlan& P, int l, const int* lo) {
    DensBox B;
    const DensLevel& Q = P.L[l - 1];
    for (int a = 0; a < 3; ++a) {
        B.pd[a] = Q.n[a];
        B.po[a] = 0;
        B.lo[a] = lo[a];
    }
    B.wrap = l == 1 ? Q.n[0] : 0;
    return B;
}

int run_density(const DensPlan& P, const double* table, double dr, int subgrid, const double* const* xi,
                double* const* delta, hipStream_t st) {
    const int top = P.nl - 1;
    // ---- kernels, finest first; each grid becomes its spectrum once the next coarser is built
    DN_HIP(launch_kernel_direct(P.L[top].T, P.L[top].D, P.L[top].h, table, dr, subgrid, st));
    for (int l = top; l >= 0; --l) {
        const DensLevel& D = P.L[l];
        if (l > 0) {
            const DensLevel& Q = P.L[l - 1];
            DN_HIP(launch_kernel_restrict(Q.T, Q.D, Q.h, D.T, D.D, table, dr, st));
        }
        DN_HIP(spec_grid_prepare(D.G, 0, 2, 4, st));
        DN_HIP(spec_forward_zy(D.G, D.T, nullptr, st));
        DN_HIP(spec_x_pass(D.G, kFftForward, kFftOutRe, 0, 1.0, nullptr, nullptr, nullptr, D.T, st));
    }
    // ---- noise: scale, refine top-down (mode replacement), then reverse Hoffman-Ribak bottom-up
    DN_HIP(launch_divide(P.L[0].mu, xi[0], cells3(P.L[0].D), std::pow(P.L[0].h, 1.5), st));
    for (int l = 1; l <= top; ++l) {
        const DensLevel& D = P.L[l];
        DN_HIP(launch_divide(D.mu, xi[l], cells3(D.D), std::pow(D.h, 1.5), st));
        int lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = D.off[a] - D.n[a] / 4;
        DN_HIP(launch_gather(P.reg, D.n, P.L[l - 1].mu, parent_box(P, l, lo), st));
        DN_HIP(spec_grid_prepare(D.R, 0, 2, 4, st));
        DN_HIP(spec_forward_zy(D.R, P.reg, nullptr, st));
        DN_HIP(spec_x_pass(D.R, kFftForward, kFftOutCplx, 0, 1.0, nullptr, nullptr, nullptr, P.csp, st));
        DN_HIP(spec_grid_prepare(D.G, kSpecReplace, 2, 4, st));
        DN_HIP(spec_forward_zy(D.G, D.mu, nullptr, st));
        DN_HIP(spec_x_pass(D.G, kFftFwdSymInv, 0, kSymReplace, 1.0, nullptr, P.csp, D.n, nullptr, st));
        DN_HIP(spec_inverse_yz(D.G, D.mu, nullptr, false, st));
    }
    for (int l = top; l >= 1; --l) {
        const DensLevel& D = P.L[l];
        const int m[3] = {D.n[0] / 2, D.n[1] / 2, D.n[2] / 2};
        const int co[3] = {D.n[0] / 2, D.n[1] / 2, D.n[2] / 2};
        DN_HIP(launch_restrict_mean(P.L[l - 1].mu, parent_box(P, l, D.off), m, D.mu, D.D, co, st));
    }
    // ---- convolutions
    {
        const DensLevel& B = P.L[0];
        DN_HIP(spec_grid_prepare(B.G, 0, 2, 4, st));
        if (top >= 1) {
            const int m[3] = {P.L[1].n[0] / 2, P.L[1].n[1] / 2, P.L[1].n[2] / 2};
            DN_HIP(launch_zero_box(P.zbase, B.mu, B.D, P.L[1].off, m, st));
            DN_HIP(spec_forward_zy(B.G, B.mu, P.zbase, st));
        } else {
            DN_HIP(spec_forward_zy(B.G, B.mu, nullptr, st));
        }
        DN_HIP(spec_x_pass(B.G, kFftFwdSymInv, 0, kSymTable, B.h * B.h * B.h, B.T, nullptr, nullptr, nullptr, st));
        DN_HIP(spec_inverse_yz(B.G, delta[0], top >= 1 ? P.carry0 : nullptr, false, st));
    }
    const double* src = P.carry0;
    double* dst = P.carryA;
    for (int l = 1; l <= top; ++l) {
        const DensLevel& D = P.L[l];
        int lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = D.off[a] - D.n[a] / 4;
        const bool next = l < top;
        int nm[3] = {0, 0, 0};
        if (next)
            for (int a = 0; a < 3; ++a) nm[a] = P.L[l + 1].n[a] / 2;
        DN_HIP(launch_conv_prep(P.a, P.b, next ? P.c : nullptr, D.mu, D.n, P.L[l - 1].mu, parent_box(P, l, lo),
                                next ? P.L[l + 1].off : nullptr, next ? nm : nullptr, st));
        DN_HIP(spec_grid_prepare(D.G, 0, 2, 4, st));
        const double v = D.h * D.h * D.h;
        DN_HIP(spec_forward_zy(D.G, P.a, P.b, st));
        DN_HIP(spec_x_pass(D.G, kFftFwdSymInv, 0, kSymTable, v, D.T, nullptr, nullptr, nullptr, st));
        DN_HIP(spec_inverse_yz(D.G, P.a, P.b, false, st));
        // coarse contributions carried down, then this level's density
        DN_HIP(launch_interp_cons(dst, D.n, src, parent_plain_box(P, l, D.off), st));
        DN_HIP(launch_patch_add(delta[l], P.a, dst, D.n, st));
        // delta_bnd restricted onto the parent cells under D' that the patch does not cover
        DN_HIP(launch_restrict_add(delta[l - 1], parent_plain_box(P, l, lo), P.b, D.n, st));
        if (next) {
            DN_HIP(spec_forward_zy(D.G, P.c, nullptr, st));
            DN_HIP(spec_x_pass(D.G, kFftFwdSymInv, 0, kSymTable, v, D.T, nullptr, nullptr, nullptr, st));
            DN_HIP(spec_inverse_yz(D.G, P.c, nullptr, false, st));
            DN_HIP(launch_patch_add(dst, P.c, dst, D.n, st));
            src = dst;
            dst = dst == P.carryA ? P.carryB : P.carryA;
        }
    }
    // ---- composite: covered coarse cells := mean of their children, finest first
    for (int l = top; l >= 1; --l) {
        const DensLevel& D = P.L[l];
        const int m[3] = {D.n[0] / 2, D.n[1] / 2, D.n[2] / 2};
        const int co[3] = {0, 0, 0};
        DN_HIP(launch_restrict_mean(delta[l - 1], parent_plain_box(P, l, D.off), m, delta[l], D.n, co, st));
    }
    return MG_OK;
}

}  // namespace

}  // namespace mgic

using namespace mgic;

extern "C" {

size_t ic_density_workspace_bytes(const mg_hier* hier) {
    DensPlan P;
    if (dens_plan(hier, nullptr, P)) return 0;
    return P.bytes;
}

int ic_multiscale_density(const mg_hier* hier, const double* radial, int nradial, double dr, int subgrid,
                          const double* const* xi, double* const* delta, void* ws, size_t ws_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    DensPlan P;
    int rc = dens_plan(hier, nullptr, P);
    if (rc) return rc;
    if (!radial || nradial < 2) return report_error(MG_EINVAL, "the radial table needs at least 2 entries");
    if (!(dr > 0) || !std::isfinite(dr)) return report_error(MG_EINVAL, "dr must be positive and finite");
    if (!xi || !delta) return report_error(MG_EINVAL, "noise or output pointer array is NULL");
    for (int l = 0; l < P.nl; ++l)
        if (!xi[l] || !delta[l]) return report_error(MG_EINVAL, "a level pointer is NULL");
    // the largest radius any kernel grid samples: the base at |D| <= sqrt(3) N/2 H, a patch's
    // padded grid at sqrt(3) n h, plus the sub-cell offsets of the finest level
    double rmax = std::sqrt(3.0) * 0.5 * P.L[0].n[0] * P.L[0].h;
    for (int l = 1; l < P.nl; ++l) {
        const DensLevel& D = P.L[l];
        const double m = (double)std::max(D.n[0], std::max(D.n[1], D.n[2]));
        rmax = std::max(rmax, std::sqrt(3.0) * m * D.h);
    }
    rmax += std::sqrt(3.0) * 0.25 * P.L[P.nl - 1].h;
    if (rmax / dr >= (double)(nradial - 2))
        return report_error(MG_EINVAL, ("the radial table must reach r = " + std::to_string(rmax)).c_str());
    if (!ws || ws_bytes < P.bytes)
        return report_error(MG_EINVAL, ("workspace too small: need " + std::to_string(P.bytes)).c_str());
    if (((uintptr_t)ws) & 255) return report_error(MG_EINVAL, "workspace must be 256-byte aligned");
    dens_plan(hier, ws, P);
    return run_density(P, radial, dr, subgrid ? 1 : 0, xi, delta, st);
}

}  // extern "C"
