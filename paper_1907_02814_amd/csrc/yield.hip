// yield.hip -- expected photon-energy yield and its adjoint.
//
// Y_c = sum_j w_j P_j <k>_j,  P = 1 - exp(-x),  x = n_i sigma_B(gamma) beta c dt,
// each electron against the ions of its cell at rest (eq:proba1) with
// n_i = n_e/Z* (Sec. II.A), <k> = sigma_k/sigma_B from the tables.
// The adjoint recomputes every lookup (nothing is stored by the forward) and
// chains through the screening state: n_i, r_i and L_D (eq:LDH), eta_D,
// I_TFD (eq:ITFD) and the reduced length, whose implicit derivative from
// eq:reduit is d ln L_R / d a = ((x+1)/x)^2, x = L_R^2.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "wave.hpp"

namespace cmc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <int kW>
__device__ double ysum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < kW; ++i) s += red[i];
    __syncthreads();
    return s;
}

// 1 - exp(-x) for x >= 0: the series to x^6 below 2^-10, where it is
// -expm1(-x) to within an ulp (the next term is below 2^-70 x), else
// -expm1(-x).
__device__ __forceinline__ double one_minus_exp(double x) {
    if (x < 0x1p-10)
        return x * (1.0 - x * (0.5 - x * (1.0 / 6 - x * (1.0 / 24 - x * (1.0 / 120 - x * (1.0 / 720))))));
    return -expm1(-x);
}

// an electron record (momenta and weight)
struct YRec { double x, y, z, w; };

// A copy in registers of its own (an instruction the compiler cannot fold),
// so that the registers a record arrived in may take the next load at once
__device__ __forceinline__ double fresh(double v) {
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ YRec fresh(const YRec& r) { return YRec{fresh(r.x), fresh(r.y), fresh(r.z), fresh(r.w)}; }

// 1/v in the form's precision: v holds an R value
template <typename R>
__device__ __forceinline__ double rcp_r(double v) {
    if constexpr (sizeof(R) == 4) return (double)__builtin_amdgcn_rcpf((float)v);
    else return 1.0 / v;
}

struct YArgs {
    const double *Zs, *ne, *Te, *px, *py, *pz, *w, *gY;
    const int64_t* off;
    double *Y, *yp, *gpx, *gpy, *gpz, *gw, *gZs, *gne, *gTe;
    int32_t* status;
    int64_t n_cells, n_part;
    double dt;
};

// The per-cell checks of the inputs: offsets inside [0, n_part] and
// non-decreasing (else nothing of the cell is touched), and a cell state
// the screening model covers: 0 < Z* <= Z, n_e > 0, T_e >= 0, all finite.
enum : int { kCellOk = 0, kCellBad = 1, kCellBadOffsets = 2 };

__device__ __forceinline__ int check_cell(int64_t j0, int64_t j1, int64_t n_part, double Zs, double ne, double Te,
                                          double Z) {
    if (!(j0 >= 0 && j1 >= j0 && j1 <= n_part)) return kCellBadOffsets;
    if (!(Zs > 0.0 && Zs <= Z && ne > 0.0 && Te >= 0.0 && isfinite(ne) && isfinite(Te))) return kCellBad;
    return kCellOk;
}

__device__ __forceinline__ void flag_cell(int32_t* status, int why) {
    if (status) atomicOr(status, why == kCellBadOffsets ? CMC_ST_BAD_OFFSETS : CMC_ST_BAD_CELL);
}

// Position of an electron on the Bremsstrahlung energy axes: segment
// (g <= 2 non-relativistic on ln(g - 1), g <= 100 relativistic, ultra-
// relativistic above, no emission at or below 1 keV; Sec. II.B), slice node
// i0 of the bracketing interval, weight w and `in` (false when clamped at
// an end of the axis), by the arithmetic of brems_lookup.  In FP32, `near`
// reports a position that the FP64 energy may place differently: within
// kKnotTol node spacings of a knot (where the slope of the interpolant
// changes), or within a few FP32 ulps of a segment join (where the cross
// section jumps), of the 1 keV floor or of the table top.
constexpr double kKnotTol = 1e-4;

template <typename A>
struct EPos { int seg, i0; A w; bool in; };

template <typename A, bool kKnots = true>
__device__ __forceinline__ EPos<A> epos(const Axes& ax, A g, A gm1, bool& near) {
    EPos<A> o{kSegNone, 0, (A)0, false};
    near = false;
    constexpr bool f32 = sizeof(A) == 4;
    const A rt = (A)4e-6;
    const A tmin = (A)(grid::kTminEv / grid::kMec2Ev);
    if (f32 && fabs(gm1 - tmin) <= rt * tmin) near = true;
    if (!(gm1 > tmin)) return o;
    // the segment's axis by value (selects of kernel arguments: a pointer
    // chosen per lane would be read from memory, and each such read waits
    // for every load in flight)
    A u, u0, du;
    int base, n;
    if (g <= (A)2) {
        o.seg = kSegNR; u0 = (A)ax.nr.u0; du = (A)ax.nr.du; n = ax.nr.n; base = 0;
        u = Fast<A>::log(gm1);
    } else if (g <= (A)100) {
        o.seg = kSegRel; u0 = (A)ax.rel.u0; du = (A)ax.rel.du; n = ax.rel.n; base = grid::kNR;
        u = Fast<A>::log(g);
    } else {
        o.seg = kSegUR; u0 = (A)ax.ur.u0; du = (A)ax.ur.du; n = ax.ur.n; base = grid::kNR + grid::kRel;
        u = g > (A)grid::kTop ? (A)log(grid::kTop) : Fast<A>::log(g);
    }
    if (f32 && (fabs(g - (A)2) <= rt * (A)2 || fabs(g - (A)100) <= rt * (A)100 ||
                fabs(g - (A)grid::kTop) <= rt * (A)grid::kTop))
        near = true;
    const A pos = Fast<A>::div(u - u0, du);
    int ig;
    if (pos <= (A)0) { ig = 0; o.w = (A)0; o.in = false; }
    else if (pos >= (A)(n - 1)) { ig = n - 2; o.w = (A)1; o.in = false; }
    else {
        ig = (int)pos;
        if (ig > n - 2) ig = n - 2;
        o.w = pos - (A)ig; o.in = true;
    }
    if (f32 && kKnots) {
        const A fr = pos - floor(pos);
        if (fr < (A)kKnotTol || fr > (A)(1.0 - kKnotTol)) near = true;
    }
    o.i0 = base + ig;
    return o;
}

// The position in the arithmetic of the form R; in FP32 it is taken again
// from the FP64 energy (momenta as stored) when the FP32 one is near a
// segment join, the floor or the top, and (kKnots, for the slopes of the
// adjoint) near a knot.  The forward needs no knots: the interpolant is
// continuous there, so either interval gives its value.
template <typename R, bool kKnots = true>
__device__ __forceinline__ EPos<R> electron_pos(const Axes& ax, R g, R gm1, double qx, double qy, double qz) {
    bool near;
    EPos<R> o = epos<R, kKnots>(ax, g, gm1, near);
    if constexpr (sizeof(R) == 4) {
        if (near) {
            const double p2 = qx * qx + qy * qy + qz * qz, gd = sqrt(1.0 + p2), gm1d = p2 / (gd + 1.0);
            bool nd;
            const EPos<double> e = epos<double>(ax, gd, gm1d, nd);
            o.seg = e.seg; o.i0 = e.i0; o.w = (R)e.w; o.in = e.in;
        }
    }
    return o;
}

// Per-cell slices of the Bremsstrahlung tables, staged in LDS once per
// cell: the screening blend of sigma_B and sigma_k at every energy node of
// the three segments (NR | rel | UR, as slice_node_brems), in the form's
// arithmetic R.  An electron's lookup then only interpolates the slices
// along energy, with the operations of brems_lookup, so its values are the
// same.
template <typename R>
__device__ __forceinline__ void yield_slice_node(const TabView<R>& T, const CellTab<R>& c, int i, R* sS, R* sK) {
    if (i < grid::kNR) {
        sS[i] = blend_N<R>(T[grid::kSigN], 1, i, c, 0);
        sK[i] = blend_N<R>(T[grid::kSkN], 1, i, c, 0);
        return;
    }
    const bool rel = i < grid::kNR + grid::kRel;
    const int ig = rel ? i - grid::kNR : i - grid::kNR - grid::kRel;
    sS[i] = blend_L<R>(T[rel ? grid::kSigR : grid::kSigU], 1, ig, c, 0);
    sK[i] = blend_L<R>(T[rel ? grid::kSkR : grid::kSkU], 1, ig, c, 0);
}

// The slopes of the interpolant for the adjoint, per slice node i, always
// from the FP64 tables (a difference of two neighbouring FP32 values would
// keep few digits where the cross section is flat): along energy, the
// slope of the interval [i, i + 1] of its segment (dS, dK; unused at a
// segment's last node), and at node i the slopes along ln L (ln L_D on the
// NR segment; sa, ka) and along eta_D (NR; se, ke), by the interpolation's
// own arithmetic.
__device__ __forceinline__ void yield_slope_node(const TabView<double>& T, const CellTab<double>& c, int i,
                                                 double* dS, double* dK, double* sa, double* ka, double* se,
                                                 double* ke) {
    const double dLn = T.ax.L.du;
    if (i < grid::kNR) {
        if (i + 1 < grid::kNR) {
            dS[i] = (blend_N<double>(T[grid::kSigN], 1, i + 1, c, 0) - blend_N<double>(T[grid::kSigN], 1, i, c, 0)) / T.ax.nr.du;
            dK[i] = (blend_N<double>(T[grid::kSkN], 1, i + 1, c, 0) - blend_N<double>(T[grid::kSkN], 1, i, c, 0)) / T.ax.nr.du;
        } else {
            dS[i] = 0.0; dK[i] = 0.0;
        }
        const double dEn = T.ax.eta.du;
        for (int q = 0; q < 2; ++q) {
            const double* TS = T[q ? grid::kSkN : grid::kSigN];
            const double* p = TS + ((size_t)i * grid::kEta + c.iE) * grid::kL + c.iD;
            const double* r = p + grid::kL;
            const double v0 = lerp(p[0], p[1], c.wD), v1 = lerp(r[0], r[1], c.wD);
            const double sl = c.inD ? lerp(p[1] - p[0], r[1] - r[0], c.wE) / dLn : 0.0;
            const double sv = c.inE ? (v1 - v0) / dEn : 0.0;
            if (q) { ka[i] = sl; ke[i] = sv; } else { sa[i] = sl; se[i] = sv; }
        }
        return;
    }
    const bool rel = i < grid::kNR + grid::kRel;
    const int ig = rel ? i - grid::kNR : i - grid::kNR - grid::kRel;
    const int n = rel ? grid::kRel : grid::kUR;
    const double du = rel ? T.ax.rel.du : T.ax.ur.du;
    const double* TS = T[rel ? grid::kSigR : grid::kSigU];
    const double* TK = T[rel ? grid::kSkR : grid::kSkU];
    if (ig + 1 < n) {
        dS[i] = (blend_L<double>(TS, 1, ig + 1, c, 0) - blend_L<double>(TS, 1, ig, c, 0)) / du;
        dK[i] = (blend_L<double>(TK, 1, ig + 1, c, 0) - blend_L<double>(TK, 1, ig, c, 0)) / du;
    } else {
        dS[i] = 0.0; dK[i] = 0.0;
    }
    const double* p = TS + (size_t)ig * grid::kL + c.iL;
    const double* r = TK + (size_t)ig * grid::kL + c.iL;
    sa[i] = c.inL ? (p[1] - p[0]) / dLn : 0.0;
    ka[i] = c.inL ? (r[1] - r[0]) / dLn : 0.0;
    se[i] = 0.0;
    ke[i] = 0.0;
}

// Bremsstrahlung lookup of an electron at position e from the slices, with
// the slopes of the interpolant when dS != nullptr: along energy (u =
// ln(g - 1) on the NR segment, ln g above) and along the screening axes
template <typename R>
struct BremsGrad {
    int seg;
    double sig, sk, ds_du, dk_du, ds_a, dk_a, ds_e, dk_e;
};

template <typename R>
__device__ __forceinline__ BremsGrad<R> brems_grad(const EPos<R>& e, const R* sS, const R* sK, const double* dS,
                                                  const double* dK, const double* sa, const double* ka,
                                                  const double* se, const double* ke) {
    BremsGrad<R> o = {};
    o.seg = e.seg;
    if (e.seg == kSegNone) return o;
    const int i0 = e.i0;
    o.sig = (double)lerp(sS[i0], sS[i0 + 1], e.w);
    o.sk = (double)lerp(sK[i0], sK[i0 + 1], e.w);
    if (dS) {
        const double w = (double)e.w;
        o.ds_du = e.in ? dS[i0] : 0.0;
        o.dk_du = e.in ? dK[i0] : 0.0;
        o.ds_a = sa[i0] + w * (sa[i0 + 1] - sa[i0]);
        o.dk_a = ka[i0] + w * (ka[i0 + 1] - ka[i0]);
        o.ds_e = se[i0] + w * (se[i0 + 1] - se[i0]);
        o.dk_e = ke[i0] + w * (ke[i0 + 1] - ke[i0]);
    }
    return o;
}

struct CellJac {
    double dlnLr[3], deta[3], dlnLd[3], dlnni[3];
};

__device__ CellJac cell_jacobian(const phys::Screen& s, double Z, double Zs, double ne, double Te) {
    CellJac J = {};
    J.dlnni[0] = -1.0 / Zs; J.dlnni[1] = 1.0 / ne;
    J.deta[0] = 1.0 / Z;
    if (s.branch == 1) {        // L_D^2 = eps0 T/(e n_e (Z* + 1))
        J.dlnLd[0] = -0.5 / (Zs + 1.0); J.dlnLd[1] = -0.5 / ne; J.dlnLd[2] = 0.5 / Te;
    } else if (s.branch == 2) { // L_D = r_i = (3 Z*/(4 pi n_e))^(1/3)
        J.dlnLd[0] = 1.0 / (3.0 * Zs); J.dlnLd[1] = -1.0 / (3.0 * ne);
    }
    const double B = s.Ld * s.Ld;
    const double X = phys::screen_cross(s.Ltf, s.Ld);
    const double da_deta = -s.eta_tf * phys::screen_self(s.Ltf) + s.eta_d * phys::screen_self(s.Ld)
                         + (s.eta_tf - s.eta_d) * X;
    const double da_dlnLd = s.eta_d * s.eta_d * B * B / ((1.0 + B) * (1.0 + B))
                          + s.eta_tf * s.eta_d * 2.0 * B * phys::screen_cross_dB(s.Ltf, s.Ld);
    const double x = s.Lr * s.Lr;
    const double dlr_da = ((x + 1.0) / x) * ((x + 1.0) / x);
    for (int q = 0; q < 3; ++q) J.dlnLr[q] = dlr_da * (da_deta * J.deta[q] + da_dlnLd * J.dlnLd[q]);
    return J;
}

// One workgroup per cell.  The first electron of each thread is in flight
// while thread 0 computes the cell's screening state; the slices are then
// staged, and every electron is evaluated with the next one's record in
// flight.  The FP32 form runs four wavefronts per SIMD (four cells per CU,
// 1024 cells in one round), the FP64 form three.
template <typename R>
__global__ __launch_bounds__(kThreads, sizeof(R) == 4 ? 4 : 3) void k_yield(YArgs A, TabView<R> T) {
    __shared__ double red[kWaves];
    __shared__ CellTab<R> ct_s;
    __shared__ R sS[kSliceBrems], sK[kSliceBrems];
    for (int64_t c = blockIdx.x; c < A.n_cells; c += gridDim.x) {
        const double Zs = A.Zs[c], ne = A.ne[c], Te = A.Te[c];
        const double ni = ne / Zs;
        const int64_t j0 = A.off[c], j1 = A.off[c + 1];
        const int bad = check_cell(j0, j1, A.n_part, Zs, ne, Te, T.Z);
        if (bad) {
            if (threadIdx.x == 0) { A.Y[c] = 0.0; flag_cell(A.status, bad); }
            if (bad == kCellBad && A.yp)
                for (int64_t j = j0 + threadIdx.x; j < j1; j += kThreads) A.yp[j] = 0.0;
            continue;
        }
        // the first two records of each thread are in flight while thread 0
        // computes the cell's screening state (reads clamped into the cell)
        const int64_t j = j0 + threadIdx.x;
        const bool any = j1 > j0;
        const auto load = [&](int64_t k) {
            const int64_t q = k < j1 ? k : j1 - 1;
            return YRec{A.px[q], A.py[q], A.pz[q], A.w[q]};
        };
        YRec ra{}, rb{};
        if (any) { ra = load(j); rb = load(j + kThreads); }
        if (threadIdx.x == 0) ct_s = cell_tab<R>(phys::screening(T.Z, Zs, ni, Te), T.ax);
        __syncthreads();
        {
            const CellTab<R> ct = ct_s;
            for (int i = threadIdx.x; i < kSliceBrems; i += kThreads) yield_slice_node<R>(T, ct, i, sS, sK);
        }
        __syncthreads();
        double acc = 0.0;
        const auto eval = [&](int64_t k, const YRec& r) {
            if (k >= j1) return;
            const R px = (R)r.x, py = (R)r.y, pz = (R)r.z;
            const R p2 = px * px + py * py + pz * pz;
            const R g = Fast<R>::sqrt((R)1 + p2), gm1 = Fast<R>::div(p2, g + (R)1);
            const EPos<R> e = electron_pos<R, false>(T.ax, g, gm1, r.x, r.y, r.z);
            const BremsGrad<R> L = brems_grad<R>(e, sS, sK, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
            double y = 0.0;
            if (L.sig > 0.0) {
                const double beta = (double)Fast<R>::div(Fast<R>::sqrt(p2), g);
                const double x = ni * L.sig * beta * phys::kC * A.dt;
                const double P = one_minus_exp(x);
                y = r.w * P * (L.sk * rcp_r<R>(L.sig));
            }
            if (A.yp) A.yp[k] = y;
            acc += y;
        };
        // two records in flight, each in registers of its own: a record is
        // copied out (fresh) before the load two ahead goes into its
        // registers (moving a value still in flight waits for every load)
        if (any) {
            for (int64_t k = j; k < j1; k += 2 * kThreads) {
                const YRec ca = fresh(ra);
                ra = load(k + 2 * kThreads);
                eval(k, ca);
                const YRec cb = fresh(rb);
                rb = load(k + 3 * kThreads);
                eval(k + kThreads, cb);
            }
        }
        const double s = ysum<kWaves>(acc, red);
        if (threadIdx.x == 0) A.Y[c] = s;
        __syncthreads();
    }
}

// Three wavefronts per SIMD (the electron loop holds more registers than
// four would leave), and workgroups of three wavefronts: a CU then holds
// four cells at once, so that 256 CUs take 1024 cells in one round.  Thread
// 0 computes the cell's screening state and lookup positions while thread 64
// computes the same state and its Jacobian, which is read only after the
// electron loop: the two serial parts run side by side.  The slopes of the
// interpolant come from the FP64 tables in both forms (T64), and the FP32
// form locates an electron near a knot from its FP64 energy, so that both
// forms differentiate the interval the FP64 energy falls in.
constexpr int kBwdThreads = 192;
template <typename R>
__global__ __launch_bounds__(kBwdThreads, 3) void k_yield_bwd(YArgs A, TabView<R> T, TabView<double> T64) {
    constexpr int kThreads = kBwdThreads;
    __shared__ double red[kThreads / 64];
    __shared__ CellTab<R> ct_s;
    __shared__ CellTab<double> ct64_s;
    __shared__ CellJac J_s;
    __shared__ R sS[kSliceBrems], sK[kSliceBrems];
    __shared__ double dS[kSliceBrems], dK[kSliceBrems];
    __shared__ double sa[kSliceBrems], ka[kSliceBrems], se[kSliceBrems], ke[kSliceBrems];
    for (int64_t c = blockIdx.x; c < A.n_cells; c += gridDim.x) {
        const double Zs = A.Zs[c], ne = A.ne[c], Te = A.Te[c], gY = A.gY[c];
        const double ni = ne / Zs;
        const int64_t j0 = A.off[c], j1 = A.off[c + 1];
        const int bad = check_cell(j0, j1, A.n_part, Zs, ne, Te, T.Z);
        if (bad) {
            if (threadIdx.x < 3) (threadIdx.x == 0 ? A.gZs : threadIdx.x == 1 ? A.gne : A.gTe)[c] = 0.0;
            if (threadIdx.x == 0) flag_cell(A.status, bad);
            if (bad == kCellBad)
                for (int64_t j = j0 + threadIdx.x; j < j1; j += kThreads) {
                    A.gpx[j] = 0.0; A.gpy[j] = 0.0; A.gpz[j] = 0.0;
                    if (A.gw) A.gw[j] = 0.0;
                }
            continue;
        }
        int64_t j = j0 + threadIdx.x;
        double nx = 0.0, ny = 0.0, nz = 0.0, nw = 0.0;
        if (j < j1) { nx = A.px[j]; ny = A.py[j]; nz = A.pz[j]; nw = A.w[j]; }
        if (threadIdx.x == 0) {
            const phys::Screen sc = phys::screening(T.Z, Zs, ni, Te);
            ct_s = cell_tab<R>(sc, T.ax);
            if constexpr (sizeof(R) == 4) ct64_s = cell_tab<double>(sc, T.ax);
        } else if (threadIdx.x == 64) {
            J_s = cell_jacobian(phys::screening(T.Z, Zs, ni, Te), T.Z, Zs, ne, Te);
        }
        __syncthreads();
        {
            const CellTab<R> ct = ct_s;
            CellTab<double> c64;
            if constexpr (sizeof(R) == 4) c64 = ct64_s; else c64 = ct;
            for (int i = threadIdx.x; i < kSliceBrems; i += kThreads) {
                yield_slice_node<R>(T, ct, i, sS, sK);
                yield_slope_node(T64, c64, i, dS, dK, sa, ka, se, ke);
            }
        }
        __syncthreads();
        // The cell gradients are linear in the cell's Jacobian: dx/dq and
        // dK/dq of an electron are n_i and the screening slopes times
        // d ln n_i/dq, d ln L_D/dq (NR segment), d ln L_R/dq (above) and
        // d eta_D/dq.  The electrons' coefficients of these four are summed,
        // and the Jacobian applied once per cell.
        double a0 = 0.0, aD = 0.0, aR = 0.0, aE = 0.0;
        for (; j < j1; j += kThreads) {
            const double qx = nx, qy = ny, qz = nz, w = nw;
            if (j + kThreads < j1) {
                nx = A.px[j + kThreads]; ny = A.py[j + kThreads]; nz = A.pz[j + kThreads]; nw = A.w[j + kThreads];
            }
            const R px = (R)qx, py = (R)qy, pz = (R)qz;
            const R p2 = px * px + py * py + pz * pz;
            const R g = Fast<R>::sqrt((R)1 + p2), gm1 = Fast<R>::div(p2, g + (R)1);
            const EPos<R> e = electron_pos<R>(T.ax, g, gm1, qx, qy, qz);
            const BremsGrad<R> L = brems_grad<R>(e, sS, sK, dS, dK, sa, ka, se, ke);
            double gx = 0.0, gyv = 0.0, gz = 0.0, gwj = 0.0;
            if (L.sig > 0.0) {
                const double gd = (double)g, beta = (double)Fast<R>::div(Fast<R>::sqrt(p2), g);
                const double x = ni * L.sig * beta * phys::kC * A.dt;
                // P' = exp(-x) = 1 - P, without cancellation for x < 1/2
                const double P = one_minus_exp(x), Pp = x < 0.5 ? 1.0 - P : exp(-x);
                const double is = rcp_r<R>(L.sig), K = L.sk * is, igd = rcp_r<R>(gd);
                const double du_dg = L.seg == kSegNR ? rcp_r<R>((double)gm1) : igd;
                const double dsig = L.ds_du * du_dg, dsk = L.dk_du * du_dg;
                const double dbeta = igd * igd * igd * rcp_r<R>(beta);
                const double dx = ni * phys::kC * A.dt * (dsig * beta + L.sig * dbeta);
                const double dK = (dsk - K * dsig) * is;
                const double f = gY * (w * (Pp * dx * K + P * dK)) * igd;
                gx = f * qx; gyv = f * qy; gz = f * qz;
                gwj = gY * P * K;
                // d(w P K)/dq = w (P' dx/dq K + P dK/dq), dx/dq = x d ln n_i/dq +
                // n_i beta c dt dsig/dq, dK/dq = dsk/dq / sig - sk dsig/dq / sig^2
                const double gw_ = gY * w;
                const double c1 = gw_ * (Pp * K * ni * beta * phys::kC * A.dt - P * K * is);
                const double c2 = gw_ * P * is;
                a0 += gw_ * Pp * K * x;
                const double ta = c1 * L.ds_a + c2 * L.dk_a;
                if (L.seg == kSegNR) {
                    aD += ta;
                    aE += c1 * L.ds_e + c2 * L.dk_e;
                } else {
                    aR += ta;
                }
            }
            A.gpx[j] = gx; A.gpy[j] = gyv; A.gpz[j] = gz;
            if (A.gw) A.gw[j] = gwj;
        }
        const double s0 = ysum<kThreads / 64>(a0, red), sD = ysum<kThreads / 64>(aD, red);
        const double sR = ysum<kThreads / 64>(aR, red), sE = ysum<kThreads / 64>(aE, red);
        if (threadIdx.x < 3) {
            const CellJac& J = J_s;
            const int q = threadIdx.x;
            const double gq = s0 * J.dlnni[q] + sD * J.dlnLd[q] + sR * J.dlnLr[q] + sE * J.deta[q];
            (q == 0 ? A.gZs : q == 1 ? A.gne : A.gTe)[c] = gq;
        }
        __syncthreads();
    }
}

int ygrid(int64_t n) { return (int)(n < 65536 ? (n > 0 ? n : 1) : 65536); }

}  // namespace
}  // namespace cmc

using namespace cmc;

static cmc_status yield_common(cmc_tables t, int64_t n_cells, const double* Zs, const double* ne,
                               const double* Te, const int64_t* off, int64_t n_part, const double* px,
                               const double* py, const double* pz, const double* w, double dt,
                               int32_t precision, const char* who) {
    CMC_REQUIRE(t, CMC_EINVAL, "%s: tables is NULL", who);
    CMC_REQUIRE(n_cells >= 0, CMC_EINVAL, "%s: n_cells < 0", who);
    CMC_REQUIRE(n_part >= 0, CMC_EINVAL, "%s: n_part < 0", who);
    CMC_REQUIRE(dt > 0.0, CMC_EINVAL, "%s: dt must be > 0", who);
    CMC_REQUIRE(precision == CMC_FP64 || precision == CMC_FP32, CMC_EINVAL, "%s: unknown precision", who);
    // with no cell nothing is read or written: the arrays may be NULL
    CMC_REQUIRE(n_cells == 0 || (Zs && ne && Te && off), CMC_EINVAL, "%s: NULL cell array", who);
    CMC_REQUIRE(n_cells == 0 || n_part == 0 || (px && py && pz && w), CMC_EINVAL, "%s: NULL particle array", who);
    CMC_REQUIRE(aligned_to<double>(Zs) && aligned_to<double>(ne) && aligned_to<double>(Te) &&
                    aligned_to<int64_t>(off) && aligned_to<double>(px) && aligned_to<double>(py) &&
                    aligned_to<double>(pz) && aligned_to<double>(w),
                CMC_EINVAL, "%s: an input array is not aligned to its element type", who);
    return CMC_OK;
}

extern "C" cmc_status cmc_expected_yield(cmc_tables t, int64_t n_cells, const double* Zstar,
                                         const double* n_e, const double* T_e, const int64_t* off,
                                         int64_t n_part, const double* px, const double* py, const double* pz,
                                         const double* w, double dt, int32_t precision, double* Y,
                                         double* y_part, int32_t* status, void* stream) {
    cmc_status s = yield_common(t, n_cells, Zstar, n_e, T_e, off, n_part, px, py, pz, w, dt, precision,
                                "cmc_expected_yield");
    if (s != CMC_OK) return s;
    if (n_cells == 0) return CMC_OK;
    CMC_REQUIRE(Y, CMC_EINVAL, "cmc_expected_yield: Y is NULL");
    CMC_REQUIRE(aligned_to<double>(Y) && aligned_to<double>(y_part) && aligned_to<int32_t>(status), CMC_EINVAL,
                "cmc_expected_yield: an output array is not aligned to its element type");
    YArgs A{};
    A.Zs = Zstar; A.ne = n_e; A.Te = T_e; A.off = off; A.px = px; A.py = py; A.pz = pz; A.w = w;
    A.Y = Y; A.yp = y_part; A.status = status; A.n_cells = n_cells; A.n_part = n_part; A.dt = dt;
    hipStream_t st = as_stream(stream);
    if (precision == CMC_FP64)
        hipLaunchKernelGGL(k_yield<double>, dim3(ygrid(n_cells)), dim3(kThreads), 0, st, A, view64(t));
    else
        hipLaunchKernelGGL(k_yield<float>, dim3(ygrid(n_cells)), dim3(kThreads), 0, st, A, view32(t));
    CMC_CHECK_LAUNCH("cmc_expected_yield");
    return CMC_OK;
}

extern "C" cmc_status cmc_expected_yield_backward(cmc_tables t, int64_t n_cells, const double* Zstar,
                                                  const double* n_e, const double* T_e,
                                                  const int64_t* off, int64_t n_part, const double* px,
                                                  const double* py, const double* pz, const double* w,
                                                  double dt, int32_t precision, const double* gY,
                                                  double* gpx, double* gpy, double* gpz, double* gw,
                                                  double* gZstar, double* gn_e, double* gT_e,
                                                  int32_t* status, void* stream) {
    cmc_status s = yield_common(t, n_cells, Zstar, n_e, T_e, off, n_part, px, py, pz, w, dt, precision,
                                "cmc_expected_yield_backward");
    if (s != CMC_OK) return s;
    if (n_cells == 0) return CMC_OK;
    CMC_REQUIRE(gY && gZstar && gn_e && gT_e, CMC_EINVAL, "cmc_expected_yield_backward: NULL output");
    CMC_REQUIRE(n_part == 0 || (gpx && gpy && gpz), CMC_EINVAL, "cmc_expected_yield_backward: NULL output");
    CMC_REQUIRE(aligned_to<double>(gY) && aligned_to<double>(gpx) && aligned_to<double>(gpy) &&
                    aligned_to<double>(gpz) && aligned_to<double>(gw) && aligned_to<double>(gZstar) &&
                    aligned_to<double>(gn_e) && aligned_to<double>(gT_e) && aligned_to<int32_t>(status),
                CMC_EINVAL, "cmc_expected_yield_backward: an array is not aligned to its element type");
    YArgs A{};
    A.Zs = Zstar; A.ne = n_e; A.Te = T_e; A.off = off; A.px = px; A.py = py; A.pz = pz; A.w = w;
    A.gY = gY; A.gpx = gpx; A.gpy = gpy; A.gpz = gpz; A.gw = gw; A.gZs = gZstar; A.gne = gn_e;
    A.gTe = gT_e; A.status = status; A.n_cells = n_cells; A.n_part = n_part; A.dt = dt;
    hipStream_t st = as_stream(stream);
    if (precision == CMC_FP64)
        hipLaunchKernelGGL(k_yield_bwd<double>, dim3(ygrid(n_cells)), dim3(kBwdThreads), 0, st, A, view64(t),
                           view64(t));
    else
        hipLaunchKernelGGL(k_yield_bwd<float>, dim3(ygrid(n_cells)), dim3(kBwdThreads), 0, st, A, view32(t),
                           view64(t));
    CMC_CHECK_LAUNCH("cmc_expected_yield_backward");
    return CMC_OK;
}
