// Host side of the spectral operations (Section 3.5 of Hahn & Abel 2011): the finite-volume and
// sub-grid deconvolutions and the hybrid Poisson correction on the finest grid, built on the
// three-pass FFT of k_fft.hip.
//
// Pipeline for a real field f of n0 x n1 x n2 cells transformed on P0 x P1 x P2 points (P = n on
// periodic grids, the zero-padded isolated length otherwise), z contiguous:
//   z pass   f            -> W1 [n0][n1][P2]   (lines zero-extended from n2 to P2)
//   y pass   W1           -> W2 [n0][P1][P2]
//   x pass   W2 -> forward, multiplier, inverse -> W3 [n0][P1][P2]   (one launch)
//   y pass   W3 (inverse) -> W1 [n0][n1][P2]
//   z pass   W1 (inverse) -> real output [n0][n1][n2]
// Only the first n points of each axis are ever stored: lines that are zero by padding are not
// transformed, and output points outside the patch are not computed past the axis they lie on.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "spec_internal.h"
#include "mgic.h"

namespace mgic {

namespace {

#define SP_HIP(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            return report_error(MG_EHIP, (std::string(#call) + ": " + hipGetErrorString(e_)).c_str()); \
        }                                                                                        \
    } while (0)

int pad_len(int n) {
    int p = 1;
    while (p < 2 * n) p *= 2;
    return p;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

FftPass pass_base(const SpecGrid& S, int axis) {
    FftPass A;
    A.lgN = S.lg[axis];
    A.lgnl = fft_lines_per_tile(A.lgN);
    A.lgtw = S.lgtw;
    A.tw = S.tw;
    return A;
}

struct SpecPlan {
    SpecGrid G;
    size_t bytes = 0;
};

// validates the shape and carves the workspace (ws == nullptr: sizes only)
int spec_plan(const int* n, int isolated, void* ws, SpecPlan& S) {
    int rc = spec_grid_init(n, isolated, S.G);
    if (rc) return rc;
    size_t off = 0;
    spec_grid_carve(S.G, (char*)ws, off);
    size_t w1, w2;
    spec_grid_work(S.G, w1, w2);
    char* base = (char*)ws;
    auto take = [&](size_t bytes) -> void* {
        off = align256(off);
        void* p = base ? (void*)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    S.G.W1 = (double2*)take(sizeof(double2) * w1);
    S.G.W2 = (double2*)take(sizeof(double2) * w2);
    S.G.W3 = (double2*)take(sizeof(double2) * w2);
    S.bytes = align256(off);
    return MG_OK;
}

int check_ws(const SpecPlan& S, void* ws, size_t ws_bytes) {
    if (!ws || ws_bytes < S.bytes)
        return report_error(MG_EINVAL, ("workspace too small: need " + std::to_string(S.bytes)).c_str());
    if (((uintptr_t)ws) & 255) return report_error(MG_EINVAL, "workspace must be 256-byte aligned");
    return MG_OK;
}

}  // namespace

int spec_grid_init(const int* n, int isolated, SpecGrid& S) {
    if (!n) return report_error(MG_EINVAL, "shape is NULL");
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1) return report_error(MG_EINVAL, "every axis needs at least one cell");
        const int P = isolated ? pad_len(n[a]) : n[a];
        const int lg = log2_exact(P);
        if (lg < 1 || lg > kFftMaxLgN)
            return report_error(MG_EINVAL, isolated ? "isolated transforms need n <= 512 on every axis"
                                                    : "periodic transforms need power-of-two n in 2..1024");
        S.n[a] = n[a];
        S.P[a] = P;
        S.lg[a] = lg;
    }
    S.lgtw = std::max(S.lg[0], std::max(S.lg[1], S.lg[2]));
    return MG_OK;
}

void spec_grid_carve(SpecGrid& S, char* base, size_t& off) {
    auto take = [&](size_t bytes) -> void* {
        off = align256(off);
        void* p = base ? (void*)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    S.tw = (double2*)take(sizeof(double2) << S.lgtw);
    for (int a = 0; a < 3; ++a) S.tab[a] = (double*)take(4 * sizeof(double) * (size_t)S.P[a]);
}

void spec_grid_work(const SpecGrid& S, size_t& w1, size_t& w2) {
    w1 = (size_t)S.n[0] * S.n[1] * S.P[2];
    w2 = (size_t)S.n[0] * S.P[1] * S.P[2];
}

hipError_t spec_grid_prepare(const SpecGrid& S, int kind, int lap_order, int grad_order, hipStream_t st) {
    hipError_t e = launch_fft_twiddles(S.tw, S.lgtw, st);
    if (e != hipSuccess) return e;
    if (kind == 0) return hipSuccess;
    return launch_spec_tables(S.tab[0], S.tab[1], S.tab[2], S.P, kind, lap_order, grad_order, st);
}

// z then y forward passes of a real field (in1 != nullptr: a second real field as the imaginary
// part) into W2
hipError_t spec_forward_zy(const SpecGrid& S, const double* in0, const double* in1, hipStream_t st) {
    FftPass z = pass_base(S, 2);
    z.na = S.n[0] * S.n[1];
    z.m_in = S.n[2];
    z.m_out = S.P[2];
    z.in_sa = S.n[2];
    z.out_sa = S.P[2];
    z.in0 = in0;
    z.in1 = in1;
    z.out0 = S.W1;
    hipError_t e = launch_fft_pass(z, true, in1 ? kFftInRePair : kFftInRe, kFftOutCplx, kFftForward, 0, st);
    if (e != hipSuccess) return e;
    FftPass y = pass_base(S, 1);
    y.na = S.n[0];
    y.nb = S.P[2];
    y.m_in = S.n[1];
    y.m_out = S.P[1];
    y.in_sa = (long long)S.n[1] * S.P[2];
    y.in_si = S.P[2];
    y.out_sa = (long long)S.P[1] * S.P[2];
    y.out_si = S.P[2];
    y.in0 = S.W1;
    y.out0 = S.W2;
    return launch_fft_pass(y, false, kFftInCplx, kFftOutCplx, kFftForward, 0, st);
}

// x pass on W2.  op kFftFwdSymInv: forward, multiply (sym), inverse, the first n0 points of every
// line into W3.  op kFftForward: the spectrum itself (every point) into out, complex
// (out_kind kFftOutCplx) or its real part (kFftOutRe), layout [P0][P1][P2].
hipError_t spec_x_pass(const SpecGrid& S, int op, int out_kind, int sym, double scale, const double* tab,
                       const double2* csp, const int* cn, void* out, hipStream_t st) {
    FftPass x = pass_base(S, 0);
    x.na = S.P[1];
    x.nb = S.P[2];
    x.m_in = S.n[0];
    x.m_out = op == kFftFwdSymInv ? S.n[0] : S.P[0];
    x.in_sa = S.P[2];
    x.in_si = (long long)S.P[1] * S.P[2];
    x.out_sa = S.P[2];
    x.out_si = x.in_si;
    x.in0 = S.W2;
    x.out0 = op == kFftFwdSymInv ? (void*)S.W3 : out;
    x.tab_x = S.tab[0];
    x.tab_y = S.tab[1];
    x.tab_z = S.tab[2];
    for (int a = 0; a < 3; ++a) x.sym_n[a] = S.P[a];
    x.tab = tab;
    x.tab_si = (long long)S.P[1] * S.P[2];
    x.tab_sa = S.P[2];
    x.csp = csp;
    if (cn)
        for (int a = 0; a < 3; ++a) x.cn[a] = cn[a];
    // the inverse transform's 1 / (P0 P1 P2) rides on the multiplier
    x.sym_scale = scale / ((double)S.P[0] * (double)S.P[1] * (double)S.P[2]);
    return launch_fft_pass(x, false, kFftInCplx, op == kFftFwdSymInv ? kFftOutCplx : out_kind, op, sym, st);
}

// y then z inverse passes, W3 -> real output(s) [n0][n1][n2] (real part -> out0, imaginary -> out1)
hipError_t spec_inverse_yz(const SpecGrid& S, double* out0, double* out1, bool add, hipStream_t st) {
    FftPass y = pass_base(S, 1);
    y.na = S.n[0];
    y.nb = S.P[2];
    y.m_in = S.P[1];
    y.m_out = S.n[1];
    y.in_sa = (long long)S.P[1] * S.P[2];
    y.in_si = S.P[2];
    y.out_sa = (long long)S.n[1] * S.P[2];
    y.out_si = S.P[2];
    y.in0 = S.W3;
    y.out0 = S.W1;
    hipError_t e = launch_fft_pass(y, false, kFftInCplx, kFftOutCplx, kFftInverse, 0, st);
    if (e != hipSuccess) return e;
    FftPass z = pass_base(S, 2);
    z.na = S.n[0] * S.n[1];
    z.m_in = S.P[2];
    z.m_out = S.n[2];
    z.in_sa = S.P[2];
    z.out_sa = S.n[2];
    z.in0 = S.W1;
    z.out0 = out0;
    z.out1 = out1;
    return launch_fft_pass(z, true, kFftInCplx, add ? kFftOutRePairAdd : kFftOutRePairStore, kFftInverse, 0, st);
}

}  // namespace mgic

using namespace mgic;

extern "C" {

size_t spec_workspace_bytes(const int n[3], int isolated) {
    SpecPlan S;
    if (spec_plan(n, isolated, nullptr, S)) return 0;
    return S.bytes;
}

int spec_deconvolve(const int n[3], int kind, int isolated, const double* f, double* out, void* ws, size_t ws_bytes,
                    void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (kind != SPEC_FV_DECONV && kind != SPEC_SG_DECONV) return report_error(MG_EINVAL, "unknown deconvolution kind");
    if (!f || !out) return report_error(MG_EINVAL, "f or out is NULL");
    SpecPlan S;
    int rc = spec_plan(n, isolated, nullptr, S);
    if (rc) return rc;
    if ((rc = check_ws(S, ws, ws_bytes))) return rc;
    spec_plan(n, isolated, ws, S);
    const SpecGrid& G = S.G;
    SP_HIP(spec_grid_prepare(G, kind == SPEC_FV_DECONV ? kSpecFv : kSpecSg, 2, 4, st));
    SP_HIP(spec_forward_zy(G, f, nullptr, st));
    SP_HIP(spec_x_pass(G, kFftFwdSymInv, 0, kSymSeparable, 1.0, nullptr, nullptr, nullptr, nullptr, st));
    SP_HIP(spec_inverse_yz(G, out, nullptr, false, st));
    return MG_OK;
}

int spec_poisson(const int n[3], double h, int order, const double* f, double* u, void* ws, size_t ws_bytes,
                 void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (order != 2 && order != 4 && order != 6) return report_error(MG_EINVAL, "order must be 2, 4 or 6");
    if (!(h > 0) || !std::isfinite(h)) return report_error(MG_EINVAL, "h must be positive and finite");
    if (!f || !u) return report_error(MG_EINVAL, "f or u is NULL");
    SpecPlan S;
    int rc = spec_plan(n, 0, nullptr, S);
    if (rc) return rc;
    if ((rc = check_ws(S, ws, ws_bytes))) return rc;
    spec_plan(n, 0, ws, S);
    const SpecGrid& G = S.G;
    SP_HIP(spec_grid_prepare(G, kSpecPoisson, order, 4, st));
    SP_HIP(spec_forward_zy(G, f, nullptr, st));
    SP_HIP(spec_x_pass(G, kFftFwdSymInv, 0, kSymInvLap, h * h, nullptr, nullptr, nullptr, nullptr, st));
    SP_HIP(spec_inverse_yz(G, u, nullptr, false, st));
    return MG_OK;
}

int lpt_hybrid_correction(const int n[3], double h, int isolated, int lap_order, int grad_order, double scale,
                          const double* f, double* const* out3, void* ws, size_t ws_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (lap_order != 2 && lap_order != 4 && lap_order != 6)
        return report_error(MG_EINVAL, "lap_order must be 2, 4 or 6");
    if (grad_order != 4 && grad_order != 6) return report_error(MG_EINVAL, "grad_order must be 4 or 6");
    if (!(h > 0) || !std::isfinite(h)) return report_error(MG_EINVAL, "h must be positive and finite");
    if (!std::isfinite(scale)) return report_error(MG_EINVAL, "scale must be finite");
    if (!f || !out3 || !out3[0] || !out3[1] || !out3[2]) return report_error(MG_EINVAL, "f or an output is NULL");
    SpecPlan S;
    int rc = spec_plan(n, isolated, nullptr, S);
    if (rc) return rc;
    if ((rc = check_ws(S, ws, ws_bytes))) return rc;
    spec_plan(n, isolated, ws, S);
    const SpecGrid& G = S.G;
    SP_HIP(spec_grid_prepare(G, kSpecHybrid, lap_order, grad_order, st));
    SP_HIP(spec_forward_zy(G, f, nullptr, st));
    // components x and y in one complex field, then z
    SP_HIP(spec_x_pass(G, kFftFwdSymInv, 0, kSymHybridXY, scale * h, nullptr, nullptr, nullptr, nullptr, st));
    SP_HIP(spec_inverse_yz(G, out3[0], out3[1], true, st));
    SP_HIP(spec_x_pass(G, kFftFwdSymInv, 0, kSymHybridZ, scale * h, nullptr, nullptr, nullptr, nullptr, st));
    SP_HIP(spec_inverse_yz(G, out3[2], nullptr, true, st));
    return MG_OK;
}

}  // extern "C"
