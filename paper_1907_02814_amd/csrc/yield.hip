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

namespace cmc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ double ysum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) s += red[i];
    __syncthreads();
    return s;
}

struct YArgs {
    const double *Zs, *ne, *Te, *px, *py, *pz, *w, *gY;
    const int64_t* off;
    double *Y, *yp, *gpx, *gpy, *gpz, *gw, *gZs, *gne, *gTe;
    int64_t n_cells;
    double dt;
};

// Bremsstrahlung lookup with the slopes of the interpolant
template <typename R>
struct BremsGrad {
    int seg;
    bool in;
    double sig, sk, ds_du, dk_du, ds_a, dk_a, ds_e, dk_e;
};

template <typename R>
__device__ BremsGrad<R> brems_grad(const TabView<R>& T, const CellTab<R>& c, R g, R gm1) {
    BremsGrad<R> o = {};
    bool high;
    const BremsLook<R> L = brems_lookup<R>(T, c, g, gm1, high);
    o.seg = L.seg; o.in = L.in;
    o.sig = (double)L.sig; o.sk = (double)L.sk;
    if (L.seg == kSegNone) return o;
    const double dLn = T.ax.L.du;
    double s0, s1, k0, k1, as[2], ak[2], es[2], ek[2];
    if (L.seg == kSegNR) {
        const double dEn = T.ax.eta.du;
        for (int h = 0; h < 2; ++h) {
            for (int q = 0; q < 2; ++q) {
                const R* TS = T[q ? grid::kSkN : grid::kSigN];
                const R* p = TS + ((size_t)(L.ig + h) * grid::kEta + c.iE) * grid::kL + c.iD;
                const R* r = p + grid::kL;
                const double v0 = (double)lerp(p[0], p[1], c.wD), v1 = (double)lerp(r[0], r[1], c.wD);
                const double sl = c.inD ? (double)lerp(p[1] - p[0], r[1] - r[0], c.wE) / dLn : 0.0;
                const double se = c.inE ? (v1 - v0) / dEn : 0.0;
                if (q) { ak[h] = sl; ek[h] = se; } else { as[h] = sl; es[h] = se; }
            }
        }
        s0 = (double)blend_N<R>(T[grid::kSigN], 1, L.ig, c, 0); s1 = (double)blend_N<R>(T[grid::kSigN], 1, L.ig + 1, c, 0);
        k0 = (double)blend_N<R>(T[grid::kSkN], 1, L.ig, c, 0); k1 = (double)blend_N<R>(T[grid::kSkN], 1, L.ig + 1, c, 0);
    } else {
        const bool rel = L.seg == kSegRel;
        const R* TS = T[rel ? grid::kSigR : grid::kSigU];
        const R* TK = T[rel ? grid::kSkR : grid::kSkU];
        for (int h = 0; h < 2; ++h) {
            const R* p = TS + (size_t)(L.ig + h) * grid::kL + c.iL;
            const R* r = TK + (size_t)(L.ig + h) * grid::kL + c.iL;
            as[h] = c.inL ? (double)(p[1] - p[0]) / dLn : 0.0;
            ak[h] = c.inL ? (double)(r[1] - r[0]) / dLn : 0.0;
            es[h] = 0.0; ek[h] = 0.0;
        }
        s0 = (double)blend_L<R>(TS, 1, L.ig, c, 0); s1 = (double)blend_L<R>(TS, 1, L.ig + 1, c, 0);
        k0 = (double)blend_L<R>(TK, 1, L.ig, c, 0); k1 = (double)blend_L<R>(TK, 1, L.ig + 1, c, 0);
    }
    const double du = L.seg == kSegNR ? T.ax.nr.du : (L.seg == kSegRel ? T.ax.rel.du : T.ax.ur.du);
    const double wg = (double)L.wg;
    o.ds_du = L.in ? (s1 - s0) / du : 0.0;
    o.dk_du = L.in ? (k1 - k0) / du : 0.0;
    o.ds_a = as[0] + wg * (as[1] - as[0]);
    o.dk_a = ak[0] + wg * (ak[1] - ak[0]);
    o.ds_e = es[0] + wg * (es[1] - es[0]);
    o.dk_e = ek[0] + wg * (ek[1] - ek[0]);
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

template <typename R>
__global__ __launch_bounds__(kThreads) void k_yield(YArgs A, TabView<R> T) {
    __shared__ double red[kWaves];
    __shared__ CellTab<R> ct_s;
    for (int64_t c = blockIdx.x; c < A.n_cells; c += gridDim.x) {
        const double Zs = A.Zs[c], ne = A.ne[c], Te = A.Te[c];
        const double ni = ne / Zs;
        if (threadIdx.x == 0) ct_s = cell_tab<R>(phys::screening(T.Z, Zs, ni, Te), T.ax);
        __syncthreads();
        const CellTab<R> ct = ct_s;
        double acc = 0.0;
        for (int64_t j = A.off[c] + threadIdx.x; j < A.off[c + 1]; j += kThreads) {
            const R px = (R)A.px[j], py = (R)A.py[j], pz = (R)A.pz[j];
            const R p2 = px * px + py * py + pz * pz;
            const R g = sqrt((R)1 + p2), gm1 = p2 / (g + (R)1);
            bool high;
            const BremsLook<R> L = brems_lookup<R>(T, ct, g, gm1, high);
            double y = 0.0;
            if (L.sig > (R)0) {
                const double beta = (double)(sqrt(p2) / g);
                const double x = ni * (double)L.sig * beta * phys::kC * A.dt;
                const double P = -expm1(-x);
                y = A.w[j] * P * ((double)L.sk / (double)L.sig);
            }
            if (A.yp) A.yp[j] = y;
            acc += y;
        }
        const double s = ysum(acc, red);
        if (threadIdx.x == 0) A.Y[c] = s;
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_yield_bwd(YArgs A, TabView<R> T) {
    __shared__ double red[kWaves];
    __shared__ CellTab<R> ct_s;
    __shared__ CellJac J_s;
    for (int64_t c = blockIdx.x; c < A.n_cells; c += gridDim.x) {
        const double Zs = A.Zs[c], ne = A.ne[c], Te = A.Te[c], gY = A.gY[c];
        const double ni = ne / Zs;
        if (threadIdx.x == 0) {
            const phys::Screen s = phys::screening(T.Z, Zs, ni, Te);
            ct_s = cell_tab<R>(s, T.ax);
            J_s = cell_jacobian(s, T.Z, Zs, ne, Te);
        }
        __syncthreads();
        const CellTab<R> ct = ct_s;
        const CellJac J = J_s;
        double gc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = A.off[c] + threadIdx.x; j < A.off[c + 1]; j += kThreads) {
            const double qx = A.px[j], qy = A.py[j], qz = A.pz[j], w = A.w[j];
            const R px = (R)qx, py = (R)qy, pz = (R)qz;
            const R p2 = px * px + py * py + pz * pz;
            const R g = sqrt((R)1 + p2), gm1 = p2 / (g + (R)1);
            const BremsGrad<R> L = brems_grad<R>(T, ct, g, gm1);
            double gx = 0.0, gyv = 0.0, gz = 0.0, gwj = 0.0;
            if (L.sig > 0.0) {
                const double gd = (double)g, beta = (double)(sqrt(p2) / g);
                const double x = ni * L.sig * beta * phys::kC * A.dt;
                const double P = -expm1(-x), Pp = exp(-x), K = L.sk / L.sig;
                const double du_dg = L.seg == kSegNR ? 1.0 / (double)gm1 : 1.0 / gd;
                const double dsig = L.ds_du * du_dg, dsk = L.dk_du * du_dg;
                const double dbeta = 1.0 / (gd * gd * gd * beta);
                const double dx = ni * phys::kC * A.dt * (dsig * beta + L.sig * dbeta);
                const double dK = (dsk * L.sig - L.sk * dsig) / (L.sig * L.sig);
                const double f = gY * (w * (Pp * dx * K + P * dK)) / gd;
                gx = f * qx; gyv = f * qy; gz = f * qz;
                gwj = gY * P * K;
                for (int q = 0; q < 3; ++q) {
                    double ds, dk;
                    if (L.seg == kSegNR) {
                        ds = L.ds_a * J.dlnLd[q] + L.ds_e * J.deta[q];
                        dk = L.dk_a * J.dlnLd[q] + L.dk_e * J.deta[q];
                    } else {
                        ds = L.ds_a * J.dlnLr[q];
                        dk = L.dk_a * J.dlnLr[q];
                    }
                    const double dxq = x * J.dlnni[q] + ni * beta * phys::kC * A.dt * ds;
                    const double dKq = (dk * L.sig - L.sk * ds) / (L.sig * L.sig);
                    gc[q] += gY * w * (Pp * dxq * K + P * dKq);
                }
            }
            A.gpx[j] = gx; A.gpy[j] = gyv; A.gpz[j] = gz;
            if (A.gw) A.gw[j] = gwj;
        }
        const double s0 = ysum(gc[0], red), s1 = ysum(gc[1], red), s2 = ysum(gc[2], red);
        if (threadIdx.x == 0) { A.gZs[c] = s0; A.gne[c] = s1; A.gTe[c] = s2; }
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
    CMC_REQUIRE(Zs && ne && Te && off && px && py && pz && w, CMC_EINVAL, "%s: NULL array", who);
    CMC_REQUIRE(dt > 0.0, CMC_EINVAL, "%s: dt must be > 0", who);
    CMC_REQUIRE(precision == CMC_FP64 || precision == CMC_FP32, CMC_EINVAL, "%s: unknown precision", who);
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
    CMC_REQUIRE(Y, CMC_EINVAL, "cmc_expected_yield: Y is NULL");
    if (n_cells == 0) return CMC_OK;
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
    CMC_REQUIRE(gY && gpx && gpy && gpz && gZstar && gn_e && gT_e, CMC_EINVAL,
                "cmc_expected_yield_backward: NULL output");
    if (n_cells == 0) return CMC_OK;
    YArgs A{};
    A.Zs = Zstar; A.ne = n_e; A.Te = T_e; A.off = off; A.px = px; A.py = py; A.pz = pz; A.w = w;
    A.gY = gY; A.gpx = gpx; A.gpy = gpy; A.gpz = gpz; A.gw = gw; A.gZs = gZstar; A.gne = gn_e;
    A.gTe = gT_e; A.n_cells = n_cells; A.dt = dt;
    hipStream_t st = as_stream(stream);
    if (precision == CMC_FP64)
        hipLaunchKernelGGL(k_yield_bwd<double>, dim3(ygrid(n_cells)), dim3(kThreads), 0, st, A, view64(t));
    else
        hipLaunchKernelGGL(k_yield_bwd<float>, dim3(ygrid(n_cells)), dim3(kThreads), 0, st, A, view32(t));
    CMC_CHECK_LAUNCH("cmc_expected_yield_backward");
    return CMC_OK;
}
