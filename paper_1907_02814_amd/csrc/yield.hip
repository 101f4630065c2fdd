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
    int64_t n_cells;
    double dt;
};

// Per-cell slices of the Bremsstrahlung tables, staged in LDS once per
// cell: the screening blend of sigma_B and sigma_k at every energy node of
// the three segments (NR | rel | UR, as slice_node_brems), and for the
// adjoint their slopes at each node along ln L (ln L_D on the NR segment)
// and along eta_D (NR segment), by the interpolation's own arithmetic.  An
// electron's lookup then only interpolates the slices along energy, with
// the operations of brems_lookup, so its values are the same.
template <typename R>
__device__ __forceinline__ void yield_slice_node(const TabView<R>& T, const CellTab<R>& c, int i, R* sS, R* sK,
                                                 double* sa, double* ka, double* se, double* ke) {
    const double dLn = T.ax.L.du;
    if (i < grid::kNR) {
        sS[i] = blend_N<R>(T[grid::kSigN], 1, i, c, 0);
        sK[i] = blend_N<R>(T[grid::kSkN], 1, i, c, 0);
        if (sa) {
            const double dEn = T.ax.eta.du;
            for (int q = 0; q < 2; ++q) {
                const R* TS = T[q ? grid::kSkN : grid::kSigN];
                const R* p = TS + ((size_t)i * grid::kEta + c.iE) * grid::kL + c.iD;
                const R* r = p + grid::kL;
                const double v0 = (double)lerp(p[0], p[1], c.wD), v1 = (double)lerp(r[0], r[1], c.wD);
                const double sl = c.inD ? (double)lerp(p[1] - p[0], r[1] - r[0], c.wE) / dLn : 0.0;
                const double sv = c.inE ? (v1 - v0) / dEn : 0.0;
                if (q) { ka[i] = sl; ke[i] = sv; } else { sa[i] = sl; se[i] = sv; }
            }
        }
        return;
    }
    const bool rel = i < grid::kNR + grid::kRel;
    const int ig = rel ? i - grid::kNR : i - grid::kNR - grid::kRel;
    const R* TS = T[rel ? grid::kSigR : grid::kSigU];
    const R* TK = T[rel ? grid::kSkR : grid::kSkU];
    sS[i] = blend_L<R>(TS, 1, ig, c, 0);
    sK[i] = blend_L<R>(TK, 1, ig, c, 0);
    if (sa) {
        const R* p = TS + (size_t)ig * grid::kL + c.iL;
        const R* r = TK + (size_t)ig * grid::kL + c.iL;
        sa[i] = c.inL ? (double)(p[1] - p[0]) / dLn : 0.0;
        ka[i] = c.inL ? (double)(r[1] - r[0]) / dLn : 0.0;
        se[i] = 0.0;
        ke[i] = 0.0;
    }
}

// Bremsstrahlung lookup from the slices, with the slopes of the
// interpolant when sa != nullptr: along energy (u = ln(g - 1) on the NR
// segment, ln g above) and along the screening axes
template <typename R>
struct BremsGrad {
    int seg;
    bool in;
    double sig, sk, ds_du, dk_du, ds_a, dk_a, ds_e, dk_e;
};

template <typename R>
__device__ __forceinline__ BremsGrad<R> brems_grad(const TabView<R>& T, const R* sS, const R* sK, const double* sa,
                                                  const double* ka, const double* se, const double* ke, R g, R gm1) {
    BremsGrad<R> o = {};
    if (!(gm1 > (R)(grid::kTminEv / grid::kMec2Ev))) return o;
    int base, ig;
    R wg;
    bool in;
    double du;
    if (g <= (R)2) {
        o.seg = kSegNR;
        locate<R>(Fast<R>::log(gm1), T.ax.nr, ig, wg, in);
        base = 0;
        du = T.ax.nr.du;
    } else {
        const bool rel = g <= (R)100;
        o.seg = rel ? kSegRel : kSegUR;
        R u;
        if (!rel && g > (R)grid::kTop) u = (R)log(grid::kTop); else u = Fast<R>::log(g);
        locate<R>(u, rel ? T.ax.rel : T.ax.ur, ig, wg, in);
        base = rel ? grid::kNR : grid::kNR + grid::kRel;
        du = rel ? T.ax.rel.du : T.ax.ur.du;
    }
    const int i0 = base + ig;
    o.in = in;
    o.sig = (double)lerp(sS[i0], sS[i0 + 1], wg);
    o.sk = (double)lerp(sK[i0], sK[i0 + 1], wg);
    if (sa) {
        const double s0 = (double)sS[i0], s1 = (double)sS[i0 + 1], k0 = (double)sK[i0], k1 = (double)sK[i0 + 1];
        const double w = (double)wg;
        o.ds_du = in ? (s1 - s0) / du : 0.0;
        o.dk_du = in ? (k1 - k0) / du : 0.0;
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
        const int64_t j1 = A.off[c + 1];
        int64_t j = A.off[c] + threadIdx.x;
        double nx = 0.0, ny = 0.0, nz = 0.0, nw = 0.0;
        if (j < j1) { nx = A.px[j]; ny = A.py[j]; nz = A.pz[j]; nw = A.w[j]; }
        if (threadIdx.x == 0) ct_s = cell_tab<R>(phys::screening(T.Z, Zs, ni, Te), T.ax);
        __syncthreads();
        {
            const CellTab<R> ct = ct_s;
            for (int i = threadIdx.x; i < kSliceBrems; i += kThreads)
                yield_slice_node<R>(T, ct, i, sS, sK, nullptr, nullptr, nullptr, nullptr);
        }
        __syncthreads();
        double acc = 0.0;
        for (; j < j1; j += kThreads) {
            const double qx = nx, qy = ny, qz = nz, w = nw;
            if (j + kThreads < j1) {
                nx = A.px[j + kThreads]; ny = A.py[j + kThreads]; nz = A.pz[j + kThreads]; nw = A.w[j + kThreads];
            }
            const R px = (R)qx, py = (R)qy, pz = (R)qz;
            const R p2 = px * px + py * py + pz * pz;
            const R g = Fast<R>::sqrt((R)1 + p2), gm1 = Fast<R>::div(p2, g + (R)1);
            const BremsGrad<R> L = brems_grad<R>(T, sS, sK, nullptr, nullptr, nullptr, nullptr, g, gm1);
            double y = 0.0;
            if (L.sig > 0.0) {
                const double beta = (double)Fast<R>::div(Fast<R>::sqrt(p2), g);
                const double x = ni * L.sig * beta * phys::kC * A.dt;
                const double P = one_minus_exp(x);
                y = w * P * (L.sk * rcp_r<R>(L.sig));
            }
            if (A.yp) A.yp[j] = y;
            acc += y;
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
// electron loop: the two serial parts run side by side.
constexpr int kBwdThreads = 192;
template <typename R>
__global__ __launch_bounds__(kBwdThreads, 3) void k_yield_bwd(YArgs A, TabView<R> T) {
    constexpr int kThreads = kBwdThreads;
    __shared__ double red[kThreads / 64];
    __shared__ CellTab<R> ct_s;
    __shared__ CellJac J_s;
    __shared__ R sS[kSliceBrems], sK[kSliceBrems];
    __shared__ double sa[kSliceBrems], ka[kSliceBrems], se[kSliceBrems], ke[kSliceBrems];
    for (int64_t c = blockIdx.x; c < A.n_cells; c += gridDim.x) {
        const double Zs = A.Zs[c], ne = A.ne[c], Te = A.Te[c], gY = A.gY[c];
        const double ni = ne / Zs;
        const int64_t j1 = A.off[c + 1];
        int64_t j = A.off[c] + threadIdx.x;
        double nx = 0.0, ny = 0.0, nz = 0.0, nw = 0.0;
        if (j < j1) { nx = A.px[j]; ny = A.py[j]; nz = A.pz[j]; nw = A.w[j]; }
        if (threadIdx.x == 0) {
            ct_s = cell_tab<R>(phys::screening(T.Z, Zs, ni, Te), T.ax);
        } else if (threadIdx.x == 64) {
            J_s = cell_jacobian(phys::screening(T.Z, Zs, ni, Te), T.Z, Zs, ne, Te);
        }
        __syncthreads();
        {
            const CellTab<R> ct = ct_s;
            for (int i = threadIdx.x; i < kSliceBrems; i += kThreads)
                yield_slice_node<R>(T, ct, i, sS, sK, sa, ka, se, ke);
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
            const BremsGrad<R> L = brems_grad<R>(T, sS, sK, sa, ka, se, ke, g, gm1);
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
                               const double* Te, const int64_t* off, const double* px, const double* py,
                               const double* pz, const double* w, double dt, int32_t precision,
                               const char* who) {
    CMC_REQUIRE(t, CMC_EINVAL, "%s: tables is NULL", who);
    CMC_REQUIRE(n_cells >= 0, CMC_EINVAL, "%s: n_cells < 0", who);
    CMC_REQUIRE(dt > 0.0, CMC_EINVAL, "%s: dt must be > 0", who);
    CMC_REQUIRE(precision == CMC_FP64 || precision == CMC_FP32, CMC_EINVAL, "%s: unknown precision", who);
    // with no cell nothing is read or written: the arrays may be NULL
    CMC_REQUIRE(n_cells == 0 || (Zs && ne && Te && off && px && py && pz && w), CMC_EINVAL, "%s: NULL array", who);
    return CMC_OK;
}

extern "C" cmc_status cmc_expected_yield(cmc_tables t, int64_t n_cells, const double* Zstar,
                                         const double* n_e, const double* T_e, const int64_t* off,
                                         const double* px, const double* py, const double* pz,
                                         const double* w, double dt, int32_t precision, double* Y,
                                         double* y_part, void* stream) {
    cmc_status s = yield_common(t, n_cells, Zstar, n_e, T_e, off, px, py, pz, w, dt, precision,
                                "cmc_expected_yield");
    if (s != CMC_OK) return s;
    if (n_cells == 0) return CMC_OK;
    CMC_REQUIRE(Y, CMC_EINVAL, "cmc_expected_yield: Y is NULL");
    YArgs A{};
    A.Zs = Zstar; A.ne = n_e; A.Te = T_e; A.off = off; A.px = px; A.py = py; A.pz = pz; A.w = w;
    A.Y = Y; A.yp = y_part; A.n_cells = n_cells; A.dt = dt;
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
                                                  const int64_t* off, const double* px,
                                                  const double* py, const double* pz, const double* w,
                                                  double dt, int32_t precision, const double* gY,
                                                  double* gpx, double* gpy, double* gpz, double* gw,
                                                  double* gZstar, double* gn_e, double* gT_e,
                                                  void* stream) {
    cmc_status s = yield_common(t, n_cells, Zstar, n_e, T_e, off, px, py, pz, w, dt, precision,
                                "cmc_expected_yield_backward");
    if (s != CMC_OK) return s;
    if (n_cells == 0) return CMC_OK;
    CMC_REQUIRE(gY && gpx && gpy && gpz && gZstar && gn_e && gT_e, CMC_EINVAL,
                "cmc_expected_yield_backward: NULL output");
    YArgs A{};
    A.Zs = Zstar; A.ne = n_e; A.Te = T_e; A.off = off; A.px = px; A.py = py; A.pz = pz; A.w = w;
    A.gY = gY; A.gpx = gpx; A.gpy = gpy; A.gpz = gpz; A.gw = gw; A.gZs = gZstar; A.gne = gn_e;
    A.gTe = gT_e; A.n_cells = n_cells; A.dt = dt;
    hipStream_t st = as_stream(stream);
    if (precision == CMC_FP64)
        hipLaunchKernelGGL(k_yield_bwd<double>, dim3(ygrid(n_cells)), dim3(kBwdThreads), 0, st, A, view64(t));
    else
        hipLaunchKernelGGL(k_yield_bwd<float>, dim3(ygrid(n_cells)), dim3(kBwdThreads), 0, st, A, view32(t));
    CMC_CHECK_LAUNCH("cmc_expected_yield_backward");
    return CMC_OK;
}
