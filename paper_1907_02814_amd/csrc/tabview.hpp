// tabview.hpp -- device view of the cross-section tables, table lookups and
// inverse-CDF sampling.  Templated on the arithmetic type R of the lookups
// and kinematics (double: plain form, float: FP32 form).
//
// Lookup rule (part of the tabulated method): linear interpolation, first
// along the screening axis of the cell (ln L_R; or L_D then eta_D for the
// non-relativistic segment), then along the energy axis.  Sampling inverts
// the piecewise-linear cumulative distribution blended the same way.
#pragma once
#include <hip/hip_runtime.h>

#include "grid.hpp"
#include "physics.hpp"

namespace cmc {

struct AxisDef { double u0, u1, du; int n; };

// axis constants, computed once on the host
struct Axes {
    AxisDef nr, rel, ur, bh, tri, split, L, eta;
};

template <typename R>
struct TabView {
    const R* a[grid::kNumArrays];
    Axes ax;
    double Z, Ltf, fc;
    __device__ __forceinline__ const R* operator[](int i) const { return a[i]; }
};

template <typename R>
__device__ __forceinline__ R lerp(R a, R b, R w) { return a + w * (b - a); }

// Elementary operations of the lookups and of the per-pair path.  FP64
// form: the correctly rounded operations.  FP32 form: the hardware's
// approximations (v_sqrt_f32, v_log_f32, v_rcp_f32, about 1 ulp), which its
// 1e-5 tolerance absorbs.  Every kernel goes through these, so the pass,
// event and sequential kernels see the same values.
template <typename R> struct Fast;
template <> struct Fast<double> {
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
};
template <> struct Fast<float> {
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float log(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};

// position on a uniform axis: i in [0, n-2], w in [0, 1]; `inside` false
// when clamped at an end (zero derivative there)
template <typename R>
__device__ __forceinline__ void locate(R u, const AxisDef& A, int& i, R& w, bool& inside) {
    const R pos = Fast<R>::div(u - (R)A.u0, (R)A.du);
    if (pos <= (R)0) { i = 0; w = (R)0; inside = false; return; }
    if (pos >= (R)(A.n - 1)) { i = A.n - 2; w = (R)1; inside = false; return; }
    int k = (int)pos;
    if (k > A.n - 2) k = A.n - 2;
    i = k; w = pos - (R)k; inside = true;
}

// per-cell lookup state (screening axes)
template <typename R>
struct CellTab {
    int iL, iE, iD;
    R wL, wE, wD;
    bool inL, inE, inD;
};

template <typename R>
__device__ __forceinline__ CellTab<R> cell_tab(const phys::Screen& s, const Axes& ax) {
    CellTab<R> t;
    locate<R>((R)s.lnLr, ax.L, t.iL, t.wL, t.inL);
    locate<R>((R)s.eta_d, ax.eta, t.iE, t.wE, t.inE);
    const double lnLd = s.eta_d > 0.0 ? log(s.Ld) : log(grid::kLmin);
    locate<R>((R)lnLd, ax.L, t.iD, t.wD, t.inD);
    return t;
}

// blend along ln L of a (energy, L) array at energy node i, column col
template <typename R>
__device__ __forceinline__ R blend_L(const R* T, int stride, int i, const CellTab<R>& c, int col) {
    const R* p = T + ((size_t)i * grid::kL + c.iL) * stride + col;
    return lerp(p[0], p[stride], c.wL);
}

// blend along ln L_D then eta_D of an (energy, eta, L) array
template <typename R>
__device__ __forceinline__ R blend_N(const R* T, int stride, int i, const CellTab<R>& c, int col) {
    const R* p = T + (((size_t)i * grid::kEta + c.iE) * grid::kL + c.iD) * stride + col;
    const R* q = p + (size_t)grid::kL * stride;
    return lerp(lerp(p[0], p[stride], c.wD), lerp(q[0], q[stride], c.wD), c.wE);
}

enum Seg { kSegNone = 0, kSegNR = 1, kSegRel = 2, kSegUR = 3 };

template <typename R>
struct BremsLook {
    int seg, ig;
    R wg;
    bool in;
    R sig, sk;
};

// Bremsstrahlung segment and cross section of an electron (gamma g,
// kinetic g1m1 = g - 1).  Regimes of Sec. II.B: g <= 2 non-relativistic,
// 2 < g <= 100 moderately relativistic, g > 100 ultra-relativistic; no
// emission below 1 keV; energies above the table are clamped (high = true).
template <typename R, bool kMoment = true>
__device__ __forceinline__ BremsLook<R> brems_lookup(const TabView<R>& T, const CellTab<R>& c,
                                                     R g, R g1m1, bool& high) {
    BremsLook<R> o;
    high = false;
    o.seg = kSegNone; o.ig = 0; o.wg = (R)0; o.in = false; o.sig = (R)0; o.sk = (R)0;
    if (!(g1m1 > (R)(grid::kTminEv / grid::kMec2Ev))) return o;
    if (g <= (R)2) {
        o.seg = kSegNR;
        locate<R>(Fast<R>::log(g1m1), T.ax.nr, o.ig, o.wg, o.in);
        const R s0 = blend_N<R>(T[grid::kSigN], 1, o.ig, c, 0), s1 = blend_N<R>(T[grid::kSigN], 1, o.ig + 1, c, 0);
        o.sig = lerp(s0, s1, o.wg);
        if (kMoment) {
            const R k0 = blend_N<R>(T[grid::kSkN], 1, o.ig, c, 0), k1 = blend_N<R>(T[grid::kSkN], 1, o.ig + 1, c, 0);
            o.sk = lerp(k0, k1, o.wg);
        }
        return o;
    }
    const bool rel = g <= (R)100;
    o.seg = rel ? kSegRel : kSegUR;
    R u;
    if (!rel && g > (R)grid::kTop) { high = true; u = (R)log(grid::kTop); } else { u = Fast<R>::log(g); }
    locate<R>(u, rel ? T.ax.rel : T.ax.ur, o.ig, o.wg, o.in);
    const R* S = T[rel ? grid::kSigR : grid::kSigU];
    o.sig = lerp(blend_L<R>(S, 1, o.ig, c, 0), blend_L<R>(S, 1, o.ig + 1, c, 0), o.wg);
    if (kMoment) {
        const R* K = T[rel ? grid::kSkR : grid::kSkU];
        o.sk = lerp(blend_L<R>(K, 1, o.ig, c, 0), blend_L<R>(K, 1, o.ig + 1, c, 0), o.wg);
    }
    return o;
}

// Bethe-Heitler total cross section at photon energy k (ion frame): zero
// at k <= 2, linear to zero below the first node (k - 2 < 1e-6), clamped
// above the table.
template <typename R>
__device__ __forceinline__ R bh_lookup(const TabView<R>& T, const CellTab<R>& c, R k,
                                       int& ik, R& wk, bool& high) {
    high = false; ik = 0; wk = (R)0;
    if (!(k > (R)2)) return (R)0;
    R x = k - (R)2;
    if (k > (R)grid::kTop) { high = true; x = (R)(grid::kTop - 2.0); }
    const R* S = T[grid::kSigB];
    if (x < (R)grid::kBHx0) return blend_L<R>(S, 1, 0, c, 0) * Fast<R>::div(x, (R)grid::kBHx0);
    bool in;
    locate<R>(Fast<R>::log(x), T.ax.bh, ik, wk, in);
    return lerp(blend_L<R>(S, 1, ik, c, 0), blend_L<R>(S, 1, ik + 1, c, 0), wk);
}

// ------------------------------------------------------------------ per-cell slices
// The screening blend of a cross-section array at every energy node of one
// cell, staged once per cell: a lookup then only interpolates the slice
// along energy.  Same operations in the same order as brems_lookup and
// bh_lookup, so the results are identical.
constexpr int kSliceBrems = grid::kNR + grid::kRel + grid::kUR;   // NR | rel | UR nodes
constexpr int kSliceBH = grid::kBH;

template <typename R>
__device__ __forceinline__ R slice_node_brems(const TabView<R>& T, const CellTab<R>& c, int i) {
    if (i < grid::kNR) return blend_N<R>(T[grid::kSigN], 1, i, c, 0);
    i -= grid::kNR;
    if (i < grid::kRel) return blend_L<R>(T[grid::kSigR], 1, i, c, 0);
    return blend_L<R>(T[grid::kSigU], 1, i - grid::kRel, c, 0);
}

template <typename R>
__device__ __forceinline__ R slice_node_bh(const TabView<R>& T, const CellTab<R>& c, int i) {
    return blend_L<R>(T[grid::kSigB], 1, i, c, 0);
}

// Bremsstrahlung sigma of an electron from the cell's slice (regimes and
// clamping as brems_lookup)
template <typename R>
__device__ __forceinline__ R brems_sig_slice(const TabView<R>& T, const R* sl, R g, R g1m1, bool& high) {
    high = false;
    if (!(g1m1 > (R)(grid::kTminEv / grid::kMec2Ev))) return (R)0;
    int ig; R wg; bool in;
    if (g <= (R)2) {
        locate<R>(Fast<R>::log(g1m1), T.ax.nr, ig, wg, in);
        return lerp(sl[ig], sl[ig + 1], wg);
    }
    const bool rel = g <= (R)100;
    R u;
    if (!rel && g > (R)grid::kTop) { high = true; u = (R)log(grid::kTop); } else { u = Fast<R>::log(g); }
    locate<R>(u, rel ? T.ax.rel : T.ax.ur, ig, wg, in);
    const R* s = sl + (rel ? grid::kNR : grid::kNR + grid::kRel);
    return lerp(s[ig], s[ig + 1], wg);
}

// Bethe-Heitler sigma of a photon from the cell's slice (as bh_lookup)
template <typename R>
__device__ __forceinline__ R bh_sig_slice(const TabView<R>& T, const R* sl, R k, bool& high) {
    high = false;
    if (!(k > (R)2)) return (R)0;
    R x = k - (R)2;
    if (k > (R)grid::kTop) { high = true; x = (R)(grid::kTop - 2.0); }
    if (x < (R)grid::kBHx0) return sl[0] * Fast<R>::div(x, (R)grid::kBHx0);
    int ik; R wk; bool in;
    locate<R>(Fast<R>::log(x), T.ax.bh, ik, wk, in);
    return lerp(sl[ik], sl[ik + 1], wk);
}

// ------------------------------------------------------------------ sampling
// blended CDF value j of the rows at energy nodes i, i+1 (kind: 0 (g, L),
// 1 (g, eta, L), 2 one-dimensional)
template <typename R>
__device__ __forceinline__ R cdf_value(const R* T, int kind, int i, R w, const CellTab<R>& c, int j) {
    R a, b;
    if (kind == 0) { a = blend_L<R>(T, grid::kRow, i, c, j); b = blend_L<R>(T, grid::kRow, i + 1, c, j); }
    else if (kind == 1) { a = blend_N<R>(T, grid::kRow, i, c, j); b = blend_N<R>(T, grid::kRow, i + 1, c, j); }
    else { a = T[(size_t)i * grid::kRow + j]; b = T[(size_t)(i + 1) * grid::kRow + j]; }
    return lerp(a, b, w);
}

// one row of a blended CDF table: array, blend kind (0 (g, L), 1 (g, eta,
// L), 2 one-dimensional), energy node i and weight w
template <typename R>
struct CdfRow { const R* T; int kind, i; R w; };

// t and ct = 1 - t from the row's values F_lo <= xi < F_hi at panel edges
// lo, hi = lo + 1; ct is formed from F_hi - xi so that it keeps its
// relative precision near the top of the row (the spectrum tip, where a
// product's gamma - 1 is small)
__device__ __forceinline__ double cdf_abscissa(int lo, double flo, double fhi, double xi, double& ct) {
    const int hi = lo + 1;
    const double d = fhi - flo;
    ct = ((double)(grid::kPanels - hi) + (fhi - xi) / d) / grid::kPanels;
    return ((double)lo + (xi - flo) / d) / grid::kPanels;
}

// abscissa t in [0, 1] with F(t) = xi for the piecewise-linear blended CDF
// (values blended in R, xi and the result in FP64): bisection over the
// panel edges
template <typename R>
__device__ __forceinline__ double cdf_invert(const R* T, int kind, int i, R w, const CellTab<R>& c,
                                             double xi, double& ct) {
    int lo = 0, hi = grid::kPanels;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((double)cdf_value<R>(T, kind, i, w, c, mid) <= xi) lo = mid; else hi = mid;
    }
    const double flo = (double)cdf_value<R>(T, kind, i, w, c, lo);
    const double fhi = (double)cdf_value<R>(T, kind, i, w, c, hi);
    return cdf_abscissa(lo, flo, fhi, xi, ct);
}

// The same inversion for the requests of a whole wavefront (every lane
// calls it; lanes with has = false only help): one request at a time, the
// 65 panel-edge values are read in parallel, one per lane (and F(64) when
// needed), then the same bisection runs on them with lane shuffles, so the
// result is identical to cdf_invert with one round of table reads instead
// of seven dependent ones.
template <typename R>
__device__ __forceinline__ double cdf_invert_wave(bool has, const CdfRow<R>& row, const CellTab<R>& c,
                                                  double xi, double& ct) {
    const int lane = (int)(threadIdx.x & 63u);
    double t = 0.0;
    unsigned long long pend = __ballot(has);
    while (pend) {
        const int e = __ffsll((long long)pend) - 1;
        pend &= pend - 1ull;
        const R* A = reinterpret_cast<const R*>(__shfl((long long)reinterpret_cast<intptr_t>(row.T), e, 64));
        const int K = __shfl(row.kind, e, 64), I = __shfl(row.i, e, 64);
        const R Wt = __shfl(row.w, e, 64);
        const double X = __shfl(xi, e, 64);
        const double Fj = (double)cdf_value<R>(A, K, I, Wt, c, lane);
        int lo = 0, hi = grid::kPanels;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (__shfl(Fj, mid, 64) <= X) lo = mid; else hi = mid;
        }
        const double flo = __shfl(Fj, lo, 64);
        const double fhi = hi < 64 ? __shfl(Fj, hi, 64) : (double)cdf_value<R>(A, K, I, Wt, c, hi);
        double cte;
        const double te = cdf_abscissa(lo, flo, fhi, X, cte);
        if (lane == e) { t = te; ct = cte; }
    }
    return t;
}

// Sampling: the row abscissa is found from the blended CDF (table values
// in R), and the energies follow from it in FP64 (events are rare; near a
// threshold gamma - 1 << 1 and FP32 would lose the product momenta).  Each
// sampler is split into its row and the energies that follow from (t, ct).

// Bremsstrahlung photon energy k and the electron's g2, g2 - 1 for an
// electron (g1, g1m1) (Sec. III.A: k' sampled on (10^-7, 1) of the kinetic
// energy by inversion of the cumulative distribution, g'_ef = g'_e - k').
// Rows are in y = ln(k/g2); y_hi - y = (1-t) Y, or (1-t)^2 Y on the
// non-relativistic segment (square-root tip).
template <typename R>
__device__ __forceinline__ CdfRow<R> brems_row(const TabView<R>& T, const BremsLook<R>& L) {
    const bool nr = L.seg == kSegNR;
    return CdfRow<R>{T[nr ? grid::kCdfN : (L.seg == kSegRel ? grid::kCdfR : grid::kCdfU)], nr ? 1 : 0, L.ig, L.wg};
}

__device__ __forceinline__ void brems_energies(int seg, double g1, double g1m1, double ct, double& k, double& g2,
                                               double& g2m1) {
    const bool nr = seg == kSegNR;
    const double Y = log((g1 - grid::kCut * g1m1) / grid::kCut);
    const double dl = nr ? ct * ct * Y : ct * Y;
    const double ey = g1m1 * exp(-dl);
    g2 = g1 / (1.0 + ey);
    g2m1 = g1m1 * (-expm1(-dl)) / (1.0 + ey);
    k = ey * g2;
}

template <typename R>
__device__ __forceinline__ void brems_sample(const TabView<R>& T, const CellTab<R>& c,
                                             const BremsLook<R>& L, double g1, double g1m1, double xi,
                                             double& k, double& g2, double& g2m1) {
    const CdfRow<R> row = brems_row<R>(T, L);
    double ct;
    cdf_invert<R>(row.T, row.kind, row.i, row.w, c, xi, ct);
    brems_energies(L.seg, g1, g1m1, ct, k, g2, g2m1);
}

// Bethe-Heitler positron / electron energies for photon energy k (row in
// ln g+ over the lower half, mirrored)
template <typename R>
__device__ __forceinline__ CdfRow<R> bh_row(const TabView<R>& T, int ik, R wk) {
    return CdfRow<R>{T[grid::kCdfB], 0, ik, wk};
}

__device__ __forceinline__ void bh_energies(double k, double t, double ct, double& gp, double& gm) {
    const double V = log(0.5 * k);
    if (t <= 0.5) { gp = exp(2.0 * t * V); gm = k - gp; }
    else { gm = exp(2.0 * ct * V); gp = k - gm; }
}

template <typename R>
__device__ __forceinline__ void bh_sample(const TabView<R>& T, const CellTab<R>& c, double k, int ik,
                                          R wk, double xi, double& gp, double& gm) {
    double ct;
    const double t = cdf_invert<R>(T[grid::kCdfB], 0, ik, wk, c, xi, ct);
    bh_energies(k, t, ct, gp, gm);
}

// Trident (Sec. II.D): pair energy from the g1 row (ln g_pair on
// [2, g1 - 1]), then the positron split from the g_pair row; gfm1 = the
// electron's kinetic energy left, g1 - 1 - g_pair, from the complement.
template <typename R>
__device__ __forceinline__ CdfRow<R> trident_row(const TabView<R>& T, double g1) {
    int i; R w; bool in;
    const double ga = g1 > grid::kTop ? grid::kTop : g1;
    locate<R>((R)log(ga), T.ax.tri, i, w, in);
    return CdfRow<R>{T[grid::kCdfT], 2, i, w};
}

// pair energy and the electron's kinetic energy left; true when the pair
// is split by the tabulated shape (g_pair > 4), else g+ = g- = g_pair/2
__device__ __forceinline__ bool trident_pair(double g1m1, double t, double ct, double& gpair, double& gp,
                                             double& gm, double& gfm1) {
    const double l2 = 0.69314718055994530942;
    const double Lg = log(g1m1) - l2;
    gpair = exp(l2 + t * Lg);
    gfm1 = -g1m1 * expm1(-ct * Lg);
    if (gpair <= 4.0) { gp = 0.5 * gpair; gm = gp; return false; }
    return true;
}

template <typename R>
__device__ __forceinline__ CdfRow<R> split_row(const TabView<R>& T, double gpair) {
    int i; R w; bool in;
    const double gq = gpair > grid::kTop ? grid::kTop : gpair;
    locate<R>((R)log(gq), T.ax.split, i, w, in);
    return CdfRow<R>{T[grid::kCdfS], 2, i, w};
}

__device__ __forceinline__ void split_energies(double gpair, double t2, double ct2, double& gp, double& gm) {
    const double glo = 2.0 / (1.0 + sqrt(1.0 - 4.0 / gpair));
    const double V = log(gpair / (2.0 * glo));
    if (t2 <= 0.5) { gp = glo * exp(2.0 * t2 * V); gm = gpair - gp; }
    else { gm = glo * exp(2.0 * ct2 * V); gp = gpair - gm; }
}

template <typename R>
__device__ __forceinline__ void trident_sample(const TabView<R>& T, double g1, double g1m1, double xi1,
                                               double xi2, double& gpair, double& gp, double& gm,
                                               double& gfm1) {
    CellTab<R> none{};
    const CdfRow<R> row = trident_row<R>(T, g1);
    double ct;
    const double t = cdf_invert<R>(row.T, row.kind, row.i, row.w, none, xi1, ct);
    if (!trident_pair(g1m1, t, ct, gpair, gp, gm, gfm1)) return;
    const CdfRow<R> row2 = split_row<R>(T, gpair);
    double ct2;
    const double t2 = cdf_invert<R>(row2.T, row2.kind, row2.i, row2.w, none, xi2, ct2);
    split_energies(gpair, t2, ct2, gp, gm);
}

}  // namespace cmc
