// physics.hpp -- screened cross sections of Martinez et al. (arXiv:1907.02814)
// as host/device functions: the Thomas-Fermi-Debye screening state
// (Sec. II.A), the reduced screening length (Sec. II.B.2), the screening
// integrals I1, I2 of a single-exponential potential, and the differential
// cross sections of Bremsstrahlung (Sec. II.B), Bethe-Heitler (Sec. II.C)
// and Trident (Sec. II.D) written as integrands of the table rows.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "grid.hpp"

#define CMC_HD __host__ __device__ inline

namespace cmc {
namespace phys {

// CODATA 2018
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kRe = 2.8179403262e-15;       // classical electron radius, m
constexpr double kRc = 3.8615926796e-13;       // hbar/(m_e c), m
constexpr double kC = 299792458.0;             // m/s
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kQe = 1.602176634e-19;
constexpr double kPi = 3.14159265358979323846;
constexpr double kMec2Ev = grid::kMec2Ev;

// ---------------------------------------------------------------- Lambert W
// Principal branch, used by eq:lambert-W (the coefficient a > 0 puts the
// argument in [-1/e, 0)).  Halley's method on f(w) = w e^w - z.  For
// |z| <= 2^-7 it starts from the Taylor series of W0 about 0, whose n-th
// coefficient is (-n)^(n-1)/n!: to z^10 the remainder is below 1e-18 of w,
// so the first step already meets the tolerance.
CMC_HD double lambert_w0(double z) {
    if (z == 0.0) return 0.0;
    double w;
    if (fabs(z) <= 0x1p-7) {
        w = z * (1.0 + z * (-1.0 + z * (1.5 + z * (-8.0 / 3.0 + z * (125.0 / 24.0 + z * (-54.0 / 5.0
              + z * (16807.0 / 720.0 + z * (-16384.0 / 315.0 + z * (531441.0 / 4480.0
              + z * (-156250.0 / 567.0))))))))));
    } else if (z > -0.25 && z < 3.0) {
        w = log1p(z);
    } else if (z <= -0.25) {
        const double q = sqrt(2.0 * (2.718281828459045 * z + 1.0));
        w = -1.0 + q * (1.0 + q * (-1.0 / 3.0 + q * (11.0 / 72.0)));
    } else {
        const double lz = log(z);
        w = lz - log(lz);
    }
    for (int n = 0; n < 60; ++n) {
        const double e = exp(w);
        const double f = w * e - z;
        const double d1 = e * (w + 1.0);
        const double step = f / (d1 - 0.5 * (w + 2.0) * f / (w + 1.0));
        w -= step;
        if (fabs(step) <= 1e-17 + 4e-16 * fabs(w)) break;
    }
    return w;
}

// ---------------------------------------------------------------- screening
// one exponential in eq:ITFD / eq:IRE: ((1+L^2) ln(1+L^2) - L^2)/(1+L^2)
CMC_HD double screen_self(double L) {
    const double L2 = L * L;
    return log1p(L2) - L2 / (1.0 + L2);
}

// cross term of eq:ITFD, [Ld^2 ln(1+Ltf^2) - Ltf^2 ln(1+Ld^2)]/(Ld^2 - Ltf^2);
// near equal lengths the removable singularity is evaluated at the
// midpoint m of the squares: (A B/m^2)(ln(1+m) - m/(1+m)).
CMC_HD double screen_cross(double La, double Lb) {
    const double A = La * La, B = Lb * Lb;
    const double diff = B - A;
    if (fabs(diff) <= 1e-4 * fmax(A, B)) {
        const double m = 0.5 * (A + B);
        return (A * B / (m * m)) * (log1p(m) - m / (1.0 + m));
    }
    return (B * log1p(A) - A * log1p(B)) / diff;
}

// d(cross)/dB, B = Lb^2 (for the adjoint)
CMC_HD double screen_cross_dB(double La, double Lb) {
    const double A = La * La, B = Lb * Lb;
    const double diff = B - A;
    if (fabs(diff) <= 1e-4 * fmax(A, B)) {
        const double m = 0.5 * (A + B);
        const double h = log1p(m) - m / (1.0 + m);
        const double hp = m / ((1.0 + m) * (1.0 + m));
        return A * h / (m * m) - A * B * h / (m * m * m) + 0.5 * A * B * hp / (m * m);
    }
    return A * (log1p(diff / (1.0 + A)) - diff / (1.0 + B)) / (diff * diff);
}

// eq:ITFD with eta_TF = q_TF/q, eta_D = q_D/q
CMC_HD double itfd(double eta_tf, double eta_d, double Ltf, double Ld) {
    double a = 0.5 * eta_tf * eta_tf * screen_self(Ltf);
    if (eta_d > 0.0)
        a += 0.5 * eta_d * eta_d * screen_self(Ld) + eta_tf * eta_d * screen_cross(Ltf, Ld);
    return a;
}

// eq:lambert-W: L_R = sqrt(exp(u) - 1), u = W(-e^{-1-2a}) + 1 + 2a.  W e^W
// equals the argument, so e^u = -1/W: L_R^2 = -(1 + W)/W and
// ln L_R = (u + ln(1 + W))/2, with ln(1 + W) from its series for
// |W| <= 2^-7 (to W^8: the remainder is below 2e-20).  W = 0 (an argument
// below the double range) keeps the exponential form.
struct Reduced { double Lr, lnLr; };
CMC_HD Reduced reduced_length_log(double a) {
    const double W = lambert_w0(-exp(-(1.0 + 2.0 * a)));
    Reduced r;
    if (W == 0.0) {
        r.Lr = sqrt(expm1(1.0 + 2.0 * a));
        r.lnLr = log(r.Lr);
        return r;
    }
    const double L2 = -(1.0 + W) / W;
    r.Lr = sqrt(L2);
    if (fabs(W) <= 0x1p-7) {
        const double l1w = W * (1.0 + W * (-1.0 / 2 + W * (1.0 / 3 + W * (-1.0 / 4 + W * (1.0 / 5
                         + W * (-1.0 / 6 + W * (1.0 / 7 + W * (-1.0 / 8))))))));
        r.lnLr = 0.5 * ((W + 1.0 + 2.0 * a) + l1w);
    } else {
        r.lnLr = 0.5 * log(L2);
    }
    return r;
}
CMC_HD double reduced_length(double a) { return reduced_length_log(a).Lr; }

struct Screen {
    double Ltf, Ld;        // normalised screening lengths L/r_C
    double eta_tf, eta_d;  // q_TF/q = 1 - Z*/Z, q_D/q = Z*/Z
    double a;              // I_TFD
    double Lr, lnLr;       // reduced length and its logarithm
    int branch;            // 0: Z* = 0; 1: Debye; 2: L_D = r_i; 3: top of the L axis
};

// Sec. II.A.  T in eV (k_B T = e T); L_D bounded below by r_i =
// (3/(4 pi n_i))^(1/3); L_D/r_C capped at the top of the table axis.
CMC_HD Screen screening(double Z, double Zs, double ni, double T) {
    Screen s;
    s.Ltf = 1.0 / (cbrt(Z) * kAlpha);       // eq:LTF: a_0 Z^{-1/3} / r_C
    s.eta_d = Zs / Z;
    s.eta_tf = 1.0 - Zs / Z;
    s.Ld = 0.0;
    s.branch = 0;
    if (Zs > 0.0) {
        const double ri = cbrt(3.0 / (4.0 * kPi * ni));
        double LD = sqrt(kEps0 * T / (kQe * ni * Zs * (Zs + 1.0)));   // eq:LDH
        s.branch = 1;
        if (!(LD >= ri)) { LD = ri; s.branch = 2; }
        s.Ld = LD / kRc;
        if (s.Ld > grid::kLmax) { s.Ld = grid::kLmax; s.branch = 3; }
    }
    s.a = itfd(s.eta_tf, s.eta_d, s.Ltf, s.Ld);
    const Reduced r = reduced_length_log(s.a);
    s.Lr = r.Lr;
    s.lnLr = r.lnLr;
    return s;
}

// ---------------------------------------------------------------- I1, I2
// eq:defphi1/eq:defphi2 for one exponential (1 - F_e = L^2u^2/(1+L^2u^2)),
// i.e. the closed forms eq:deriv_I1/eq:deriv_I2, evaluated in s = L u on
// [s0, L], s0 = L delta:
//   I1 = J3 - 2 s0 J2 + s0^2 J1,
//   I2 = J3 + 3 s0^2 J1 - 4 s0^3 J0 - 6 s0^2 Jlog,
// with Jn = int s^n/(1+s^2)^2 ds and Jlog = int s ln(s/s0)/(1+s^2)^2 ds.
// J0 is the difference of upper tails, summed as a series when s0 >= 2,
// where the printed closed form cancels catastrophically.
CMC_HD double tail_j0(double s) {   // int_s^inf (1+t^2)^-2 dt, s >= 2
    const double r = 1.0 / (s * s);
    double pw = r / s, acc = 0.0;
    for (int n = 0; n < 400; ++n) {
        const double term = (double)(n + 1) / (double)(2 * n + 3) * pw;
        acc = (n & 1) ? acc - term : acc + term;
        if (term < 1e-18 * fabs(acc)) break;
        pw *= r;
    }
    return acc;
}

CMC_HD void screening_integrals(double delta, double L, double& I1, double& I2) {
    const double s0 = L * delta;
    const double L2 = L * L, s02 = s0 * s0;
    const double one_m = 1.0 - delta, one_p = 1.0 + delta;
    const double q = (1.0 + L2) * (1.0 + s02);
    const double dat = atan(L * one_m / (1.0 + L2 * delta));     // atan L - atan s0
    const double J3 = 0.5 * (log1p(L2 * one_m * one_p / (1.0 + s02)) - L2 * one_m * one_p / q);
    const double J1 = 0.5 * L2 * one_m * one_p / q;
    const double J2 = 0.5 * (dat + L * one_m * (s0 * L - 1.0) / q);
    const double J0 = (s0 < 2.0) ? 0.5 * (dat - L * one_m * (s0 * L - 1.0) / q)
                                 : tail_j0(s0) - tail_j0(L);
    const double Jlog = 0.5 * log(delta) / (1.0 + L2)
                      + 0.25 * (log1p(1.0 / s02) - log1p(1.0 / L2));
    I1 = J3 - 2.0 * s0 * J2 + s02 * J1;
    I2 = J3 + 3.0 * s02 * J1 - 4.0 * s02 * s0 * J0 - 6.0 * s02 * Jlog;
}

// f_C(Z), Sec. II.B.3, four terms: a^2 [1/(1+a^2) + sum_n (-a^2)^n (zeta(2n+3)-1)]
CMC_HD double coulomb_correction(double Z) {
    const double a2 = (kAlpha * Z) * (kAlpha * Z);
    const double z3 = 0.2020569031595942854, z5 = 0.0369277551433699263;
    const double z7 = 0.0083492773819228268, z9 = 0.0020083928260822144;
    return a2 * (1.0 / (1.0 + a2) + z3 - a2 * (z5 - a2 * (z7 - a2 * z9)));
}

// ---------------------------------------------------------------- Bremsstrahlung
// Rows in y = ln(k/g2), k in (kCut (g1-1), g1-1).  Y = y_hi - y_lo and a
// point at distance dl = y_hi - y from the spectrum tip has
//   e^y = (g1-1) e^{-dl}, g2 = g1/(1+e^y), g2-1 = (g1-1)(1-e^{-dl})/(1+e^y),
//   k = e^y g2, delta = k/(2 g1 g2) = e^y/(2 g1), dk/dy = k g2/g1.
CMC_HD double brems_span(double g1, double g1m1) {
    const double klo = grid::kCut * g1m1;
    return log((g1 - klo) / grid::kCut);
}

struct BremsPoint { double k, g2, g2m1, ey; };

CMC_HD BremsPoint brems_point(double g1, double g1m1, double dl) {
    BremsPoint b;
    b.ey = g1m1 * exp(-dl);
    b.g2 = g1 / (1.0 + b.ey);
    b.g2m1 = g1m1 * (-expm1(-dl)) / (1.0 + b.ey);
    b.k = b.ey * b.g2;
    return b;
}

// eq:csre (fc = 0) or eq:csur (fc = f_C) times dk/dy
CMC_HD double brems_rel_dy(double Z, double g1, const BremsPoint& b, double L, double fc) {
    double I1, I2;
    screening_integrals(b.ey / (2.0 * g1), L, I1, I2);
    const double r = b.g2 / g1;
    const double br = (1.0 + r * r) * (I1 + 1.0 - fc) - (2.0 / 3.0) * r * (I2 + 5.0 / 6.0 - fc);
    return 4.0 * Z * Z * kRe * kRe * kAlpha * r * br;
}

// g of eq:cs_br_nr; A = dp+^2 L^2 + 1, B = dp-^2 L^2 + 1, A - B = 4 L^2 p1 p2
CMC_HD double nr_g(double eta, double L, double dpp, double dpm, double p1p2) {
    const double L2 = L * L;
    const double A = dpp * dpp * L2 + 1.0, B = dpm * dpm * L2 + 1.0;
    const double z = 4.0 * L2 * p1p2;
    return 0.5 * eta * eta * (log1p(z / B) - z / (A * B));
}

// Gamma_c of eq:cs_br_nr
CMC_HD double nr_gamma_c(double etf, double ed, double Ltf, double Ld,
                         double dpp, double dpm, double p1p2) {
    const double A = Ltf * Ltf, B = Ld * Ld, diff = B - A;
    if (fabs(diff) <= 1e-4 * fmax(A, B)) {
        const double m = 0.5 * (A + B);
        const double Am = dpp * dpp * m + 1.0, Bm = dpm * dpm * m + 1.0;
        const double z = 4.0 * m * p1p2;
        return etf * ed * (log1p(z / Bm) - z / (Am * Bm));
    }
    const double ltf = log1p(4.0 * A * p1p2 / (dpm * dpm * A + 1.0));
    const double ld = log1p(4.0 * B * p1p2 / (dpm * dpm * B + 1.0));
    return etf * ed * (B * ltf - A * ld) / diff;
}

// eq:cs_br_nr times the Elwert factor (nuclear Z), with the kinematic
// momentum-transfer bounds p1 +- p2 (reading of the printed 2p1-k and k),
// times dk/dy.
CMC_HD double brems_nr_dy(double Z, double g1, double g1m1, const BremsPoint& b,
                          double etf, double ed, double Ltf, double Ld) {
    const double p1 = sqrt(g1m1 * (g1 + 1.0));
    const double p2 = sqrt(b.g2m1 * (b.g2 + 1.0));
    const double dpp = p1 + p2;
    const double dpm = b.k * (g1 + b.g2) / dpp;
    const double p1p2 = p1 * p2;
    double br = nr_g(etf, Ltf, dpp, dpm, p1p2);
    if (ed > 0.0) br += nr_g(ed, Ld, dpp, dpm, p1p2) + nr_gamma_c(etf, ed, Ltf, Ld, dpp, dpm, p1p2);
    const double b1 = p1 / g1, b2 = p2 / b.g2, c = 2.0 * kPi * Z * kAlpha;
    const double fe = (b1 / b2) * expm1(-c / b1) / expm1(-c / b2);
    const double dsdk = 16.0 * kRe * kRe * Z * Z * kAlpha / (3.0 * b.k * p1 * p1) * br * fe;
    return dsdk * b.k * b.g2 / g1;
}

// ---------------------------------------------------------------- Bethe-Heitler
// eq:dsdkbh with delta = k/(2 g+ g-)
CMC_HD double bh_dsdgp(double Z, double k, double gp, double L) {
    const double gm = k - gp;
    double I1, I2;
    screening_integrals(k / (2.0 * gp * gm), L, I1, I2);
    return 4.0 * Z * Z * kRe * kRe * kAlpha / (k * k * k) *
           ((gp * gp + gm * gm) * (I1 + 1.0) + (2.0 / 3.0) * gp * gm * (I2 + 5.0 / 6.0));
}

// ---------------------------------------------------------------- Trident
// Gryaznykh fit (Sec. II.D); zero where the pair range [2, g1-1] is empty
CMC_HD double trident_sigma(double Z, double g1) {
    if (!(g1 > 3.0)) return 0.0;
    const double l = log((g1 + 4.50) / 6.89);
    return 5.22e-34 * Z * Z * l * l * l;
}

// bracket of eq:ds_dEpa_part1, x = 1/g1
CMC_HD double trident_nr_bracket(double g1) {
    const double x2 = 1.0 / (g1 * g1), x4 = x2 * x2;
    const double q = x2 / (1.0 - x2), lg = -log(x2);
    const double u = q * (1.0 - q * lg);
    const double C = 4.0 * q * lg - (4.0 / 3.0) * x2 + x4 / 6.0;
    const double Cz = 3.0 * u + x2 * (-2.6 + x2 * (1.75 + x2 * (-0.9 + 0.2 * x2)));
    const double Cr = -1.5 * u + x2 * (0.8 + x2 * (-0.125 + x2 * (-0.05 + 0.025 * x2)));
    return log(g1 * g1) - 161.0 / 60.0 + C + Cr + Cz;
}

// d sigma_T/d g_pair = a b/(a + b) of the two Bhabha limits, E_p = g_p m c^2,
// C1 = C2 = 1 (Z r_e alpha)^2 dropped: only the shape is tabulated
CMC_HD double trident_pair_shape(double g1, double nrb, double gpair) {
    const double a = nrb / 32.0 * gpair * gpair * gpair;
    const double b = 56.0 / (9.0 * kPi) * log(gpair) * log(g1 / gpair) / gpair;
    return a * b / (a + b);
}

// lower edge of the positive part of Bhabha's split shape:
// g+ g- > g_pair  <=>  g+ in (g_lo, g_pair - g_lo)
CMC_HD double split_low_edge(double gpair) {
    const double q = 1.0 - 4.0 / gpair;
    return 2.0 / (1.0 + sqrt(q > 0.0 ? q : 0.0));
}

}  // namespace phys
}  // namespace cmc
