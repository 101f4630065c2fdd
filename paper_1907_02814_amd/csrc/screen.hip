// screen.hip -- the screening functions I1, I2 (eq:defphi1, eq:defphi2)
// and the cross sections built on them (eq:csre, eq:csur, eq:dsdkbh) in
// either screening form of Sec. II.B.2: the reduced potential (one
// exponential of length L_R, eq:lambert-W; the form the step uses) or the
// two-exponential Thomas-Fermi-Debye potential itself (eq:V_TFD), the
// comparison curves of Figs. 5, 7 and 8.
//
// Two exponentials: with f_X(u) = (L_X u)^2/(1 + (L_X u)^2) the form
// factor is 1 - F_e = etf f_TF + ed f_D (eq:defF), and
//   [1 - F_e]^2 = etf^2 f_TF^2 + ed^2 f_D^2 + 2 etf ed f_TF f_D.
// The squares are the one-exponential functions (closed forms
// eq:deriv_I1, eq:deriv_I2); the cross term has no elementary form for I2
// and is integrated here for both functions, in t = ln u over [ln delta, 0],
// by Gauss-Legendre on panels of at most one unit of t split at the form
// factor's scales ln(1/L_TF), ln(1/L_D).  The integrand is analytic in a
// strip of half-width pi/2 about the real t axis (the poles of f_X), so
// kGl points per unit panel leave an error far below FP64 rounding.
//
// One thread per point; no table is read (the handle gives Z and f_C(Z)).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "physics.hpp"

namespace cmc {
namespace {

constexpr int kThreads = 256;
constexpr int kGl = 16;        // Gauss-Legendre points per panel

// Nodes and weights of the kGl-point Gauss-Legendre rule on [-1, 1] into
// LDS: thread i < kGl finds root i of P_kGl by Newton's method from
// cos(pi (i + 3/4)/(kGl + 1/2)); the weight is 2/((1 - x^2) P'(x)^2).
__device__ void gl_rule(double* x, double* w) {
    const int i = threadIdx.x;
    if (i < kGl) {
        double z = cos(phys::kPi * (i + 0.75) / (kGl + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 60; ++it) {
            double p0 = 1.0, p1 = z;
            for (int n = 2; n <= kGl; ++n) {
                const double p2 = ((2 * n - 1) * z * p1 - (n - 1) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            dp = kGl * (z * p1 - p0) / (z * z - 1.0);
            const double step = p1 / dp;
            z -= step;
            if (fabs(step) <= 1e-17) {
                // P' at the converged root
                p0 = 1.0; p1 = z;
                for (int n = 2; n <= kGl; ++n) {
                    const double p2 = ((2 * n - 1) * z * p1 - (n - 1) * p0) / n;
                    p0 = p1;
                    p1 = p2;
                }
                dp = kGl * (z * p1 - p0) / (z * z - 1.0);
                break;
            }
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    __syncthreads();
}

// the cross-term integrals C1 = int (1 - delta/u)^2 f_TF f_D dt and
// C2 = int [1 - 6 q^2 ln(u/delta) + 3 q^2 - 4 q^3] f_TF f_D dt, q = delta/u
// (eq:defphi1, eq:defphi2 per unit t = ln u)
__device__ void cross_integrals(double delta, double Ltf, double Ld, const double* gx, const double* gw,
                                double& C1, double& C2) {
    const double lo = log(delta);
    double cut[4];
    int nc = 0;
    cut[nc++] = lo;
    double a = -log(Ltf), b = -log(Ld);
    if (a > b) { const double s = a; a = b; b = s; }
    if (a > lo && a < 0.0) cut[nc++] = a;
    if (b > lo && b < 0.0 && b > cut[nc - 1]) cut[nc++] = b;
    cut[nc++] = 0.0;
    const double A = Ltf * Ltf, B = Ld * Ld;
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j + 1 < nc; ++j) {
        const double t0 = cut[j], t1 = cut[j + 1];
        const int np = max(1, (int)ceil(t1 - t0));
        const double h = (t1 - t0) / np;
        for (int p = 0; p < np; ++p) {
            const double c = t0 + (p + 0.5) * h, half = 0.5 * h;
            for (int g = 0; g < kGl; ++g) {
                const double t = c + half * gx[g];
                const double u = exp(t), u2 = u * u;
                const double ff = (A * u2 / (1.0 + A * u2)) * (B * u2 / (1.0 + B * u2));
                const double q = delta / u, q2 = q * q;
                const double k1 = (1.0 - q) * (1.0 - q);
                const double k2 = 1.0 - 6.0 * q2 * (t - lo) + 3.0 * q2 - 4.0 * q2 * q;
                s1 += half * gw[g] * k1 * ff;
                s2 += half * gw[g] * k2 * ff;
            }
        }
    }
    C1 = s1;
    C2 = s2;
}

struct Pt {
    bool ok;
    phys::Screen s;
};

__device__ Pt cell_at(double Z, double Zs, double ni, double T) {
    Pt p;
    p.ok = Zs >= 0.0 && Zs <= Z && ni > 0.0 && isfinite(ni) && T >= 0.0 && isfinite(T);
    if (p.ok) p.s = phys::screening(Z, Zs, ni, T);
    return p;
}

__device__ void integrals(int form, double delta, const phys::Screen& s, const double* gx, const double* gw,
                          double& I1, double& I2) {
    if (form == CMC_SCREEN_REDUCED) {
        phys::screening_integrals(delta, s.Lr, I1, I2);
        return;
    }
    double a1, a2;
    phys::screening_integrals(delta, s.Ltf, a1, a2);
    I1 = s.eta_tf * s.eta_tf * a1;
    I2 = s.eta_tf * s.eta_tf * a2;
    if (s.eta_d > 0.0) {
        double b1, b2, c1, c2;
        phys::screening_integrals(delta, s.Ld, b1, b2);
        cross_integrals(delta, s.Ltf, s.Ld, gx, gw, c1, c2);
        I1 += s.eta_d * s.eta_d * b1 + 2.0 * s.eta_tf * s.eta_d * c1;
        I2 += s.eta_d * s.eta_d * b2 + 2.0 * s.eta_tf * s.eta_d * c2;
    }
}

struct SArgs {
    const double *Zs, *ni, *Te, *e1, *x;
    double *o1, *o2;
    int32_t* status;
    int64_t n;
    double Z, fc;
    int form, process;
};

__device__ void flag_bad(int32_t* status) {
    if (status) atomicOr(status, CMC_ST_BAD_CELL);
}

__global__ __launch_bounds__(kThreads) void k_screen_fn(SArgs A) {
    __shared__ double gx[kGl], gw[kGl];
    gl_rule(gx, gw);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * kThreads) {
        const Pt p = cell_at(A.Z, A.Zs[i], A.ni[i], A.Te[i]);
        const double d = A.x[i];
        if (!p.ok || !(d > 0.0 && d <= 1.0)) {
            A.o1[i] = NAN;
            A.o2[i] = NAN;
            flag_bad(A.status);
            continue;
        }
        double I1, I2;
        integrals(A.form, d, p.s, gx, gw, I1, I2);
        A.o1[i] = I1;
        A.o2[i] = I2;
    }
}

__global__ __launch_bounds__(kThreads) void k_cross_sections(SArgs A) {
    __shared__ double gx[kGl], gw[kGl];
    gl_rule(gx, gw);
    const double pre = 4.0 * A.Z * A.Z * phys::kRe * phys::kRe * phys::kAlpha;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * kThreads) {
        const Pt p = cell_at(A.Z, A.Zs[i], A.ni[i], A.Te[i]);
        const double e = A.e1[i], x = A.x[i];
        const bool brems = A.process == CMC_BREMS;
        const bool ok = p.ok && x > 0.0 && x < 1.0 && isfinite(e) && (brems ? e >= 2.0 : e > 2.0);
        if (!ok) {
            A.o1[i] = NAN;
            flag_bad(A.status);
            continue;
        }
        double I1, I2;
        if (brems) {
            // k dsigma/dk: eq:csre up to gamma_1 = 100, eq:csur (Coulomb-corrected) above
            const double k = x * (e - 1.0), g2 = e - k, r = g2 / e;
            const double fc = e > 100.0 ? A.fc : 0.0;
            integrals(A.form, k / (2.0 * e * g2), p.s, gx, gw, I1, I2);
            A.o1[i] = pre * ((1.0 + r * r) * (I1 + 1.0 - fc) - (2.0 / 3.0) * r * (I2 + 5.0 / 6.0 - fc));
        } else {
            // dsigma/dgamma_+: eq:dsdkbh
            const double gp = 1.0 + x * (e - 2.0), gm = e - gp;
            integrals(A.form, e / (2.0 * gp * gm), p.s, gx, gw, I1, I2);
            A.o1[i] = pre / (e * e * e) * ((gp * gp + gm * gm) * (I1 + 1.0) + (2.0 / 3.0) * gp * gm * (I2 + 5.0 / 6.0));
        }
    }
}

unsigned sgrid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 8192)); }

}  // namespace
}  // namespace cmc

using namespace cmc;

extern "C" cmc_status cmc_screening_functions(cmc_tables t, int32_t form, int64_t n, const double* Zstar,
                                              const double* n_i, const double* T_e, const double* delta,
                                              double* I1, double* I2, int32_t* status, void* stream) {
    CMC_REQUIRE(t, CMC_EINVAL, "cmc_screening_functions: tables is NULL");
    CMC_REQUIRE(form == CMC_SCREEN_REDUCED || form == CMC_SCREEN_TFD, CMC_EINVAL,
                "cmc_screening_functions: unknown form %d", form);
    CMC_REQUIRE(n >= 0, CMC_EINVAL, "cmc_screening_functions: n < 0");
    if (n == 0) return CMC_OK;
    CMC_REQUIRE(Zstar && n_i && T_e && delta && I1 && I2, CMC_EINVAL, "cmc_screening_functions: NULL array");
    CMC_REQUIRE(aligned_to<double>(Zstar) && aligned_to<double>(n_i) && aligned_to<double>(T_e) &&
                    aligned_to<double>(delta) && aligned_to<double>(I1) && aligned_to<double>(I2) &&
                    aligned_to<int32_t>(status),
                CMC_EINVAL, "cmc_screening_functions: an array is not aligned to its element type");
    SArgs A{};
    A.Zs = Zstar; A.ni = n_i; A.Te = T_e; A.x = delta; A.o1 = I1; A.o2 = I2; A.status = status; A.n = n;
    A.Z = (double)t->Z; A.fc = t->fc; A.form = form;
    hipLaunchKernelGGL(k_screen_fn, dim3(sgrid(n)), dim3(kThreads), 0, as_stream(stream), A);
    CMC_CHECK_LAUNCH("cmc_screening_functions");
    return CMC_OK;
}

extern "C" cmc_status cmc_cross_sections(cmc_tables t, int32_t process, int32_t form, int64_t n,
                                         const double* Zstar, const double* n_i, const double* T_e,
                                         const double* e1, const double* x, double* out, int32_t* status,
                                         void* stream) {
    CMC_REQUIRE(t, CMC_EINVAL, "cmc_cross_sections: tables is NULL");
    CMC_REQUIRE(process == CMC_BREMS || process == CMC_BH, CMC_EINVAL,
                "cmc_cross_sections: process must be CMC_BREMS or CMC_BH");
    CMC_REQUIRE(form == CMC_SCREEN_REDUCED || form == CMC_SCREEN_TFD, CMC_EINVAL,
                "cmc_cross_sections: unknown form %d", form);
    CMC_REQUIRE(n >= 0, CMC_EINVAL, "cmc_cross_sections: n < 0");
    if (n == 0) return CMC_OK;
    CMC_REQUIRE(Zstar && n_i && T_e && e1 && x && out, CMC_EINVAL, "cmc_cross_sections: NULL array");
    CMC_REQUIRE(aligned_to<double>(Zstar) && aligned_to<double>(n_i) && aligned_to<double>(T_e) &&
                    aligned_to<double>(e1) && aligned_to<double>(x) && aligned_to<double>(out) &&
                    aligned_to<int32_t>(status),
                CMC_EINVAL, "cmc_cross_sections: an array is not aligned to its element type");
    SArgs A{};
    A.Zs = Zstar; A.ni = n_i; A.Te = T_e; A.e1 = e1; A.x = x; A.o1 = out; A.status = status; A.n = n;
    A.Z = (double)t->Z; A.fc = t->fc; A.form = form; A.process = process;
    hipLaunchKernelGGL(k_cross_sections, dim3(sgrid(n)), dim3(kThreads), 0, as_stream(stream), A);
    CMC_CHECK_LAUNCH("cmc_cross_sections");
    return CMC_OK;
}
