/*
 * cmc_oracle.c -- plain FP64 CPU oracle for the pairwise Coulomb-process
 * Monte Carlo step (Bremsstrahlung, Bethe-Heitler, Coulomb Trident) of
 * Martinez et al., "High-Energy Radiation and Pair Production by Coulomb
 * Processes in Particle-In-Cell Simulations" (arXiv:1907.02814).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load or call
 * this file; it is the slow, sequential reference that the HIP library is
 * compared against.  It shares no code with the HIP library.
 *
 * Every function cites the passage of the paper it follows (section and
 * equation label).  Where the paper is silent or garbled the reading taken
 * is stated at the spot ("reading: ...").
 *
 * Parity status: every function here is pinned by the CPU test-suite
 * (tests/test_oracle_*.py) against closed forms, limits, quadrature of the
 * paper's integral definitions, brute force or statistics.  Philox4x32-10
 * is pinned bit for bit against rocRAND's header-only engine, an
 * independent implementation of the published generator.  The sampling
 * tables of pair production are pinned against quadrature of the
 * differential cross sections in another variable and rule, and their
 * samplers by Kolmogorov-Smirnov tests against the exact distributions.
 * The screening functions of the two-exponential potential (quadrature of
 * eq:defphi1, eq:defphi2) are pinned by the printed one-exponential forms,
 * by eq:ITFD as delta -> 0, and by a partial-fraction closed form with a
 * dilogarithm for any two exponentials.
 * The Trident formulas of Sec. II.D (Gryaznykh's fit, Bhabha's two limits
 * and their interpolation, the split shape) have no value printed in the
 * paper: their relativistic form is pinned by Racah's high-energy total,
 * the rest only by their limits, scaling and symmetry ("parity unpinned"
 * for the non-relativistic bracket as a transcription).
 */
#include "cmc_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Constants (CODATA 2018; the paper names no constant set)           */
/* ------------------------------------------------------------------ */
static const double ALPHA  = 1.0 / 137.035999084;   /* fine structure      */
static const double RE     = 2.8179403262e-15;      /* r_e, m              */
static const double RC     = 3.8615926796e-13;      /* r_C = hbar/(m_e c)  */
static const double CLIGHT = 299792458.0;
static const double EPS0   = 8.8541878128e-12;
static const double QE     = 1.602176634e-19;
static const double MEC2EV = 510998.95;
static const double PI     = 3.14159265358979323846;

/* ------------------------------------------------------------------ */
/* Table grid (the definition of the tabulated method; Sec. III.A     */
/* only says the cross sections are tabulated in the ion frame)       */
/* ------------------------------------------------------------------ */
#define M_CDF 64          /* CDF panels per table row                      */
#define NGL 8             /* Gauss-Legendre points per panel               */
#define KCUT 1.0e-7       /* photon energy cut k/(g1-1) = 10^-n, n = 7     */
#define T_MIN_EV 1000.0   /* no Bremsstrahlung below 1 keV kinetic energy  */
#define GMAX 2.0e4        /* top of every energy axis (10 GeV)             */
#define N_NR 23           /* ln(g-1) in [ln(1 keV/mc^2), 0]                */
#define N_R 56            /* ln g in [ln 2, ln 100]                        */
#define N_U 75            /* ln g in [ln 100, ln 2e4]                      */
#define N_B 166           /* ln(k-2) in [ln 1e-6, ln(2e4-2)]               */
#define N_T 124           /* ln g1 in [ln 3, ln 2e4]                       */
#define N_S 120           /* ln g_pair in [ln 4, ln 2e4]                   */
#define N_L 81            /* ln L in [ln 10, ln 1e6]                       */
#define N_ETA 17          /* eta_D in [0, 1]                               */
#define L_MIN 10.0
#define L_MAX 1.0e6
#define BH_X0 1.0e-6

struct or_tables_s {
    int Z;
    double Ltf, fc;
    double *sR, *kR, *cR;   /* [N_R][N_L], [N_R][N_L], [N_R][N_L][M+1]      */
    double *sU, *kU, *cU;   /* [N_U][N_L] ...                               */
    double *sN, *kN, *cN;   /* [N_NR][N_ETA][N_L] ...                       */
    double *sB, *cB;        /* [N_B][N_L], [N_B][N_L][M+1]                  */
    double *cT;             /* [N_T][M+1]                                    */
    double *cS;             /* [N_S][M+1]                                    */
};

static double GLX[NGL], GLW[NGL];

/* Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n. */
void or_gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

static void gl_init(void)
{
    static int done = 0;
    if (!done) { or_gauss_legendre(NGL, GLX, GLW); done = 1; }
}

/* ------------------------------------------------------------------ */
/* Screening model, Sec. II.A (eq:LTF, eq:LDH, eq:V_TFD) and          */
/* the reduced potential, Sec. II.B.2 (eq:ITFD, eq:IRE, eq:reduit,    */
/* eq:lambert-W)                                                      */
/* ------------------------------------------------------------------ */

/* Principal branch W_0 of the Lambert function, Halley iteration.
 * eq:lambert-W; reading: the principal branch (W_-1 gives x < 0). */
double or_lambert_w0(double z)
{
    if (z < -0.36787944117144233) return NAN;
    if (z == 0.0) return 0.0;
    double w;
    if (z < -0.25) {
        double p = sqrt(2.0 * (2.718281828459045 * z + 1.0));
        w = -1.0 + p - p * p / 3.0 + 11.0 / 72.0 * p * p * p;
    } else if (z < 3.0) {
        w = log1p(z);
    } else {
        double l = log(z);
        w = l - log(l);
    }
    for (int it = 0; it < 60; it++) {
        double ew = exp(w);
        double f = w * ew - z;
        double wp1 = w + 1.0;
        double dw = f / (ew * wp1 - (w + 2.0) * f / (2.0 * wp1));
        w -= dw;
        if (fabs(dw) <= 1e-17 + 4e-16 * fabs(w)) break;
    }
    return w;
}

/* ((1+L^2) ln(1+L^2) - L^2)/(1+L^2): eq:ITFD / eq:IRE for one exponential */
static double h_single(double L)
{
    double q = L * L;
    return log1p(q) - q / (1.0 + q);
}

/* cross term of eq:ITFD: [B ln(1+A) - A ln(1+B)]/(B - A), A = La^2, B = Lb^2.
 * Near A = B the divided difference is replaced by its midpoint form
 * (A B / m^2)(ln(1+m) - m/(1+m)), m = (A+B)/2 (removable singularity). */
static double itfd_cross(double La, double Lb)
{
    double A = La * La, B = Lb * Lb, D = B - A;
    double M = A > B ? A : B;
    if (fabs(D) <= 1e-4 * M) {
        double m = 0.5 * (A + B);
        return (A * B / (m * m)) * (log1p(m) - m / (1.0 + m));
    }
    return (B * log1p(A) - A * log1p(B)) / D;
}

/* eq:ITFD, with q_TF/q = etf and q_D/q = ed. */
double or_I_tfd(double etf, double ed, double Ltf, double Ld)
{
    double a = 0.5 * etf * etf * h_single(Ltf);
    if (ed > 0.0)
        a += 0.5 * ed * ed * h_single(Ld) + etf * ed * itfd_cross(Ltf, Ld);
    return a;
}

/* eq:lambert-W: reduced length from a = I_TFD. */
double or_L_reduced(double a)
{
    double W = or_lambert_w0(-exp(-1.0 - 2.0 * a));
    return sqrt(expm1(W + 1.0 + 2.0 * a));
}

/* Cell screening state.
 * out = {Ltf, Ld, etf, ed, a, Lr, branch, ri/r_C}
 * branch: 0 no Debye term (Z* = 0), 1 Debye length, 2 clamped to r_i,
 *         3 clamped to the top of the table axis (L_MAX).
 * Readings: T in eV so k_B T = T e; L_TF = a_0 Z^(-1/3) exactly as
 * eq:LTF prints it; Debye terms dropped at Z* = 0; L_D >= r_i (Sec. II.A);
 * L_D/r_C clamped to L_MAX = 1e6 (top of the screening axis; reached only
 * for Z* so small that eta_D^2 ln L_D is negligible). */
void or_screening(double Z, double Zs, double ni, double T, double out[8])
{
    double Ltf = 1.0 / (cbrt(Z) * ALPHA);
    double etf = 1.0 - Zs / Z, ed = Zs / Z;
    double Ld = 0.0, ri = cbrt(3.0 / (4.0 * PI * ni));
    double branch = 0.0;
    if (Zs > 0.0) {
        double LD = sqrt(EPS0 * T / (QE * ni * Zs * (Zs + 1.0)));
        branch = 1.0;
        if (!(LD >= ri)) { LD = ri; branch = 2.0; }
        Ld = LD / RC;
        if (Ld > L_MAX) { Ld = L_MAX; branch = 3.0; }
    }
    double a = or_I_tfd(etf, ed, Ltf, Ld);
    out[0] = Ltf; out[1] = Ld; out[2] = etf; out[3] = ed;
    out[4] = a; out[5] = or_L_reduced(a); out[6] = branch; out[7] = ri / RC;
}

/* ------------------------------------------------------------------ */
/* Screening functions I1, I2 for one exponential, eq:defphi1,       */
/* eq:defphi2 with 1 - F_e(u) = L^2 u^2/(1 + L^2 u^2) (eq:app_FT_V). */
/* The closed forms eq:deriv_I1, eq:deriv_I2 are evaluated in the     */
/* variable s = L u over [s0 = L delta, L], where                     */
/*   I1 = int s (s - s0)^2 /(1+s^2)^2 ds,                             */
/*   I2 = int [s^3 + 3 s0^2 s - 4 s0^3 - 6 s0^2 s ln(s/s0)]/(1+s^2)^2 */
/* term by term, with the upper tail of int (1+s^2)^-2 summed as a    */
/* series for s0 >= 2 (the printed form loses every digit there).     */
/* ------------------------------------------------------------------ */
static double tail_inv1ps2sq(double s)   /* int_s^inf (1+t^2)^-2 dt, s >= 2 */
{
    double x = 1.0 / (s * s), p = x / s, sum = 0.0;
    for (int n = 0; n < 400; n++) {
        double term = (n + 1.0) * p / (2.0 * n + 3.0);
        sum += (n & 1) ? -term : term;
        if (term < 1e-18 * fabs(sum)) break;
        p *= x;
    }
    return sum;
}

void or_I12(double d, double L, double* I1, double* I2)
{
    double s = L * d, L2 = L * L, s2 = s * s;
    double omd = 1.0 - d, opd = 1.0 + d;
    double den = (1.0 + L2) * (1.0 + s2);
    double at = atan(L * omd / (1.0 + L2 * d));              /* atan L - atan s */
    double A3 = 0.5 * (log1p(L2 * omd * opd / (1.0 + s2)) - L2 * omd * opd / den);
    double A2 = 0.5 * (at + L * omd * (s * L - 1.0) / den);
    double A1 = 0.5 * L2 * omd * opd / den;
    double A0;
    if (s < 2.0) A0 = 0.5 * (at + L * omd * (1.0 - s * L) / den);
    else         A0 = tail_inv1ps2sq(s) - tail_inv1ps2sq(L);
    double Alog = 0.5 * log(d) / (1.0 + L2) + 0.25 * (log1p(1.0 / s2) - log1p(1.0 / L2));
    *I1 = A3 - 2.0 * s * A2 + s2 * A1;
    *I2 = A3 + 3.0 * s2 * A1 - 4.0 * s2 * s * A0 - 6.0 * s2 * Alog;
}

/* Coulomb correction, Sec. II.B.3.  Reading: the printed sum starts at
 * zeta(1) - 1 = infinity; the four-term truncation used is
 *   f_C = a^2 [1/(1+a^2) + sum_{n=0..3} (-a^2)^n (zeta(2n+3) - 1)],
 * a = alpha Z, the expansion of a^2 sum_nu 1/(nu (nu^2 + a^2)). */
double or_fc(double Z)
{
    static const double zm1[4] = { 0.2020569031595942854, 0.0369277551433699263,
                                   0.0083492773819228268, 0.0020083928260822144 };
    double a2 = (ALPHA * Z) * (ALPHA * Z);
    double s = 1.0 / (1.0 + a2), p = 1.0;
    for (int n = 0; n < 4; n++) { s += p * zm1[n]; p *= -a2; }
    return a2 * s;
}

/* ------------------------------------------------------------------ */
/* Screening functions of the two-exponential potential eq:V_TFD       */
/* (Sec. II.B.2; the comparison curves of Figs. 5, 7 and 8):           */
/* eq:defphi1 and eq:defphi2 with the form factor of eq:defF for       */
/*   V = (q_TF/r) exp(-r/L_TF) + (q_D/r) exp(-r/L_D),                  */
/*   1 - F_e(u) = etf (Ltf u)^2/(1 + (Ltf u)^2)                        */
/*              + ed (Ld u)^2/(1 + (Ld u)^2),                          */
/* etf = q_TF/q, ed = q_D/q, lengths in units of r_C.  Computed by      */
/* quadrature of the definitions, in t = ln u over [ln delta, 0]:      */
/* panels no wider than TFD_PANEL in t, split at the form factor's     */
/* scales ln(1/Ltf) and ln(1/Ld), each with TFD_NGL-point              */
/* Gauss-Legendre.  The integrands are analytic in t within a strip of */
/* half-width pi/2, so the rule converges geometrically.               */
/* ------------------------------------------------------------------ */
#define TFD_NGL 16
#define TFD_PANEL 0.25

static double one_minus_F(double u, double etf, double ed, double Ltf, double Ld)
{
    double a = Ltf * u, v = etf * a * a / (1.0 + a * a);
    if (ed > 0.0) {
        double b = Ld * u;
        v += ed * b * b / (1.0 + b * b);
    }
    return v;
}

/* eq:defphi1 and eq:defphi2 integrands per unit t = ln u (du = u dt),
 * with r = u / delta: (u - delta)^2/u^2 G^2 and
 * [1 - 6 ln(r)/r^2 + 3/r^2 - 4/r^3] G^2. */
static void tfd_panel(double t0, double t1, double d, double etf, double ed, double Ltf, double Ld,
                      double* s1, double* s2)
{
    static double X[TFD_NGL], Wt[TFD_NGL];
    static int done = 0;
    if (!done) { or_gauss_legendre(TFD_NGL, X, Wt); done = 1; }
    double h = 0.5 * (t1 - t0), m = 0.5 * (t1 + t0);
    for (int i = 0; i < TFD_NGL; i++) {
        double t = m + h * X[i], u = exp(t), r = u / d;
        double G = one_minus_F(u, etf, ed, Ltf, Ld), G2 = G * G;
        double ir = 1.0 / r;
        double k1 = (1.0 - ir) * (1.0 - ir);
        double k2 = 1.0 - 6.0 * log(r) * ir * ir + 3.0 * ir * ir - 4.0 * ir * ir * ir;
        *s1 += h * Wt[i] * k1 * G2;
        *s2 += h * Wt[i] * k2 * G2;
    }
}

void or_I12_tfd(double d, double etf, double ed, double Ltf, double Ld, double* I1, double* I2)
{
    double s1 = 0.0, s2 = 0.0;
    double lo = log(d);
    double cut[4];
    int nc = 0;
    cut[nc++] = lo;
    double c1 = -log(Ltf), c2 = ed > 0.0 ? -log(Ld) : 0.0;
    if (c1 > c2) { double tmp = c1; c1 = c2; c2 = tmp; }
    if (c1 > lo && c1 < 0.0) cut[nc++] = c1;
    if (c2 > lo && c2 < 0.0 && c2 > cut[nc - 1]) cut[nc++] = c2;
    cut[nc++] = 0.0;
    for (int j = 0; j + 1 < nc; j++) {
        double a = cut[j], b = cut[j + 1];
        int np = (int)ceil((b - a) / TFD_PANEL);
        if (np < 1) np = 1;
        double w = (b - a) / np;
        for (int p = 0; p < np; p++) {
            double t0 = a + p * w, t1 = (p + 1 == np) ? b : a + (p + 1) * w;
            tfd_panel(t0, t1, d, etf, ed, Ltf, Ld, &s1, &s2);
        }
    }
    *I1 = s1;
    *I2 = s2;
}

/* eq:csre / eq:csur and eq:dsdkbh with the screening functions of the
 * two-exponential potential (the numerically computed TFD forms). */
double or_dsdk_rel_tfd(double Z, double g1, double k, double etf, double ed, double Ltf, double Ld, int coulomb)
{
    double g2 = g1 - k, d = k / (2.0 * g1 * g2), r = g2 / g1, I1, I2;
    double fc = coulomb ? or_fc(Z) : 0.0;
    or_I12_tfd(d, etf, ed, Ltf, Ld, &I1, &I2);
    return 4.0 * Z * Z * RE * RE * ALPHA / k
         * ((1.0 + r * r) * (I1 + 1.0 - fc) - (2.0 / 3.0) * r * (I2 + 5.0 / 6.0 - fc));
}

double or_dsdgp_bh_tfd(double Z, double k, double gp, double etf, double ed, double Ltf, double Ld)
{
    double gm = k - gp, d = k / (2.0 * gp * gm), I1, I2;
    or_I12_tfd(d, etf, ed, Ltf, Ld, &I1, &I2);
    return 4.0 * Z * Z * RE * RE * ALPHA / (k * k * k)
         * ((gp * gp + gm * gm) * (I1 + 1.0) + (2.0 / 3.0) * gp * gm * (I2 + 5.0 / 6.0));
}


/* ------------------------------------------------------------------ */
/* Bremsstrahlung differential cross sections (ion rest frame)        */
/* ------------------------------------------------------------------ */

/* g of eq:cs_br_nr with A = dp+^2 L^2 + 1, B = dp-^2 L^2 + 1, written
 * with ln(A/B) = log1p(4 L^2 p1 p2 / B), since dp+^2 - dp-^2 = 4 p1 p2. */
static double nr_g(double eta, double L, double dpp, double dpm, double p1p2)
{
    double L2 = L * L;
    double A = dpp * dpp * L2 + 1.0, B = dpm * dpm * L2 + 1.0;
    double z = 4.0 * L2 * p1p2;
    return 0.5 * eta * eta * (log1p(z / B) - z / (A * B));
}

/* Gamma_c of eq:cs_br_nr. */
static double nr_coupling(double etf, double ed, double Ltf, double Ld,
                          double dpp, double dpm, double p1p2)
{
    double A = Ltf * Ltf, B = Ld * Ld, D = B - A;
    double M = A > B ? A : B;
    if (fabs(D) <= 1e-4 * M) {
        double m = 0.5 * (A + B);
        double Am = dpp * dpp * m + 1.0, Bm = dpm * dpm * m + 1.0, z = 4.0 * m * p1p2;
        return etf * ed * (log1p(z / Bm) - z / (Am * Bm));
    }
    double ltf = log1p(4.0 * A * p1p2 / (dpm * dpm * A + 1.0));
    double ld  = log1p(4.0 * B * p1p2 / (dpm * dpm * B + 1.0));
    return etf * ed * (B * ltf - A * ld) / D;
}

/* eq:cs_br_nr times the Elwert factor (Sec. II.B.1).
 * Reading: the momentum-transfer bounds are the kinematic p1 +- p2 (the
 * printed 2 p1 - k and k do not reduce to the Born point-Coulomb form and
 * make the Elwert-corrected spectrum diverge at the tip); the Elwert Z is
 * the nuclear charge.  g1m1 = g1 - 1 and g2m1 = g2 - 1 are passed
 * separately for accuracy at low energy. */
static double nr_dsdk_core(double Z, double g1, double g1m1, double k, double g2, double g2m1,
                           double etf, double ed, double Ltf, double Ld, int elwert)
{
    double p1 = sqrt(g1m1 * (g1 + 1.0)), p2 = sqrt(g2m1 * (g2 + 1.0));
    double dpp = p1 + p2, dpm = k * (g1 + g2) / (p1 + p2), p1p2 = p1 * p2;
    double br = nr_g(etf, Ltf, dpp, dpm, p1p2);
    if (ed > 0.0)
        br += nr_g(ed, Ld, dpp, dpm, p1p2) + nr_coupling(etf, ed, Ltf, Ld, dpp, dpm, p1p2);
    double fe = 1.0;
    if (elwert) {
        double b1 = p1 / g1, b2 = p2 / g2, c = 2.0 * PI * Z * ALPHA;
        fe = (b1 / b2) * expm1(-c / b1) / expm1(-c / b2);
    }
    return 16.0 * RE * RE * Z * Z * ALPHA / (3.0 * k * p1 * p1) * br * fe;
}

double or_dsdk_nr(double Z, double g1, double k, double etd, double Ltf, double Ld, int elwert)
{
    double g2 = g1 - k;
    return nr_dsdk_core(Z, g1, g1 - 1.0, k, g2, g2 - 1.0, 1.0 - etd, etd, Ltf, Ld, elwert);
}

/* curly bracket of eq:csre (fc = 0) and eq:csur (fc = f_C(Z)), r = g2/g1 */
static double rel_bracket(double d, double L, double r, double fc)
{
    double I1, I2;
    or_I12(d, L, &I1, &I2);
    return (1.0 + r * r) * (I1 + 1.0 - fc) - (2.0 / 3.0) * r * (I2 + 5.0 / 6.0 - fc);
}

/* eq:csre / eq:csur with delta = k/(2 g1 (g1 - k)), at screening length L */
double or_dsdk_rel(double Z, double g1, double k, double L, int coulomb)
{
    double g2 = g1 - k, d = k / (2.0 * g1 * g2);
    double fc = coulomb ? or_fc(Z) : 0.0;
    return 4.0 * Z * Z * RE * RE * ALPHA / k * rel_bracket(d, L, g2 / g1, fc);
}

/* eq:dsdkbh, delta = k/(2 g+ g-). */
double or_dsdgp_bh(double Z, double k, double gp, double L)
{
    double gm = k - gp, d = k / (2.0 * gp * gm), I1, I2;
    or_I12(d, L, &I1, &I2);
    return 4.0 * Z * Z * RE * RE * ALPHA / (k * k * k)
         * ((gp * gp + gm * gm) * (I1 + 1.0) + (2.0 / 3.0) * gp * gm * (I2 + 5.0 / 6.0));
}

/* ------------------------------------------------------------------ */
/* Trident, Sec. II.D                                                  */
/* ------------------------------------------------------------------ */
/* Gryaznykh fit.  Reading: sigma_T = 0 for g1 <= 3, where the pair
 * energy range [2, g1 - 1] is empty; ln is the natural logarithm. */
double or_sigma_trident(double Z, double g1)
{
    if (!(g1 > 3.0)) return 0.0;
    double l = log((g1 + 4.50) / 6.89);
    return 5.22 * Z * Z * l * l * l * 1e-34;
}

/* bracket of eq:ds_dEpa_part1: ln g1^2 - 161/60 + C + C_r + C_z, x = 1/g1 */
static double trident_nr_bracket(double g1)
{
    double x = 1.0 / g1, x2 = x * x, x4 = x2 * x2, x6 = x4 * x2, x8 = x4 * x4;
    double q = x2 / (1.0 - x2), lg = log(1.0 / x2);
    double C  = 4.0 * q * lg - 4.0 / 3.0 * x2 + x4 / 6.0;
    double Cz = 3.0 * q * (1.0 - q * lg) - 13.0 / 5.0 * x2 + 7.0 / 4.0 * x4
              - 9.0 / 10.0 * x6 + x8 / 5.0;
    double Cr = -1.5 * q * (1.0 - q * lg) + 0.8 * x2 - x4 / 8.0 - x6 / 20.0 + x8 / 40.0;
    return log(g1 * g1) - 161.0 / 60.0 + C + Cr + Cz;
}

/* Interpolated pair-energy spectrum d sigma_T/d g_p = a b/(a + b).
 * Readings: E_p = g_p m c^2; C1 = C2 = 1; the printed product
 * "(d sigma_nr d g_p)" is the density d sigma_nr/d g_p. */
double or_dsdgp_trident(double Z, double g1, double gpair)
{
    double zra = Z * RE * ALPHA, zra2 = zra * zra;
    double a = zra2 / 32.0 * trident_nr_bracket(g1) * gpair * gpair * gpair;
    double b = 56.0 / (9.0 * PI) * zra2 * log(gpair) * log(g1 / gpair) / gpair;
    return a * b / (a + b);
}

/* Positron split shape (Bhabha's doubly differential form, Sec. II.D).
 * Reading: negative values are clipped to zero. */
double or_split_shape(double gpair, double gplus)
{
    double gm = gpair - gplus;
    double v = (gplus * gplus + gm * gm + 2.0 / 3.0 * gplus * gm) * log(gplus * gm / gpair);
    return v > 0.0 ? v : 0.0;
}

/* ------------------------------------------------------------------ */
/* Tables: for every row, M_CDF panels of the row abscissa t in [0,1], */
/* each integrated with NGL-point Gauss-Legendre; the row stores the   */
/* total, the energy moment (Bremsstrahlung) and the normalised CDF at */
/* the panel edges (numerical inversion of the cumulative, Sec. III.A).*/
/* ------------------------------------------------------------------ */
typedef struct {
    int kind;               /* 0 rel/ur Brems, 1 NR Brems, 2 BH, 3 Trident pair, 4 split */
    double Z, g1, g1m1, L, fc, etf, ed, Ltf, Ld, Y, k, V;
} rowctx;

/* log of the y = ln(k/g2) range of a Bremsstrahlung row: y_hi - y_lo
 * with k_lo = KCUT (g1 - 1), y_lo = ln(k_lo/(g1 - k_lo)), y_hi = ln(g1 - 1). */
static double brems_yrange(double g1, double g1m1)
{
    double klo = KCUT * g1m1;
    return log((g1 - klo) / KCUT);
}

/* kinematics of a Bremsstrahlung abscissa: distance dl = y_hi - y >= 0 from
 * the spectrum tip; returns k and g2, g2 - 1 accurately */
static void brems_kin(double g1, double g1m1, double dl, double* k, double* g2, double* g2m1)
{
    double ey = g1m1 * exp(-dl);
    *g2 = g1 / (1.0 + ey);
    *g2m1 = g1m1 * (-expm1(-dl)) / (1.0 + ey);
    *k = ey * (*g2);
}

static double row_integrand(const rowctx* c, double t, double* fk)
{
    *fk = 0.0;
    switch (c->kind) {
    case 0: { /* relativistic Brems in y = ln(k/g2); dk/dy = k g2/g1 */
        double dl = (1.0 - t) * c->Y, k, g2, g2m1;
        brems_kin(c->g1, c->g1m1, dl, &k, &g2, &g2m1);
        double d = (c->g1m1 * exp(-dl)) / (2.0 * c->g1);
        double r = g2 / c->g1;
        double v = 4.0 * c->Z * c->Z * RE * RE * ALPHA * r * rel_bracket(d, c->L, r, c->fc) * c->Y;
        *fk = k * v;
        return v;
    }
    case 1: { /* NR Brems in y, with y_hi - y = (1-t)^2 Y (square-root tip) */
        double dl = (1.0 - t) * (1.0 - t) * c->Y, k, g2, g2m1;
        brems_kin(c->g1, c->g1m1, dl, &k, &g2, &g2m1);
        double ds = nr_dsdk_core(c->Z, c->g1, c->g1m1, k, g2, g2m1, c->etf, c->ed, c->Ltf, c->Ld, 1);
        double v = ds * (k * g2 / c->g1) * 2.0 * (1.0 - t) * c->Y;
        *fk = k * v;
        return v;
    }
    case 2: { /* BH, lower half in v = ln g+ in [0, ln(k/2)] */
        double v = 2.0 * t * c->V, gp = exp(v);
        return or_dsdgp_bh(c->Z, c->k, gp, c->L) * gp * 2.0 * c->V;
    }
    case 3: { /* Trident pair energy in v = ln g_p in [ln 2, ln(g1 - 1)] */
        double v = log(2.0) + t * c->V, gpair = exp(v);
        return or_dsdgp_trident(c->Z, c->g1, gpair) * gpair * c->V;
    }
    default: { /* split, lower half in v = ln(g+/g_lo) in [0, ln(gp/(2 g_lo))] */
        double glo = c->L, gpair = c->k;
        double v = 2.0 * t * c->V, gplus = glo * exp(v), gminus = gpair - gplus;
        double lg = log1p(glo * expm1(v) * (gpair - glo - gplus) / gpair);
        return (gplus * gplus + gminus * gminus + 2.0 / 3.0 * gplus * gminus) * lg * gplus * 2.0 * c->V;
    }
    }
}

static void build_row(const rowctx* c, int half, double* sig, double* sk, double* cdf)
{
    double C[M_CDF + 1], Ck = 0.0;
    int np = half ? M_CDF / 2 : M_CDF;
    C[0] = 0.0;
    for (int j = 0; j < np; j++) {
        double acc = 0.0, acck = 0.0;
        for (int g = 0; g < NGL; g++) {
            double t = (j + 0.5 * (1.0 + GLX[g])) / M_CDF, fk;
            double v = row_integrand(c, t, &fk);
            acc += GLW[g] * v;
            acck += GLW[g] * fk;
        }
        C[j + 1] = C[j] + acc * (0.5 / M_CDF);
        Ck += acck * (0.5 / M_CDF);
    }
    double total = half ? 2.0 * C[M_CDF / 2] : C[M_CDF];
    if (!(total > 0.0)) {
        for (int j = 0; j <= M_CDF; j++) cdf[j] = (double)j / M_CDF;
        total = 0.0; Ck = 0.0;
    } else if (half) {
        for (int j = 0; j <= M_CDF / 2; j++) cdf[j] = C[j] / total;
        for (int j = M_CDF / 2 + 1; j <= M_CDF; j++) cdf[j] = 1.0 - C[M_CDF - j] / total;
    } else {
        for (int j = 0; j <= M_CDF; j++) cdf[j] = C[j] / total;
    }
    if (sig) *sig = total;
    if (sk) *sk = Ck;
}

static double axis_node(double u0, double u1, int n, int i)
{
    return u0 + i * ((u1 - u0) / (n - 1));
}

int or_tables_build(int Z, or_tables** out)
{
    if (Z < 1 || Z > 100 || !out) return 1;
    gl_init();
    or_tables* t = (or_tables*)calloc(1, sizeof(or_tables));
    if (!t) return 2;
    t->Z = Z;
    t->Ltf = 1.0 / (cbrt((double)Z) * ALPHA);
    t->fc = or_fc((double)Z);
    const int R1 = M_CDF + 1;
    t->sR = calloc((size_t)N_R * N_L, 8);  t->kR = calloc((size_t)N_R * N_L, 8);
    t->cR = calloc((size_t)N_R * N_L * R1, 8);
    t->sU = calloc((size_t)N_U * N_L, 8);  t->kU = calloc((size_t)N_U * N_L, 8);
    t->cU = calloc((size_t)N_U * N_L * R1, 8);
    t->sN = calloc((size_t)N_NR * N_ETA * N_L, 8); t->kN = calloc((size_t)N_NR * N_ETA * N_L, 8);
    t->cN = calloc((size_t)N_NR * N_ETA * N_L * R1, 8);
    t->sB = calloc((size_t)N_B * N_L, 8);  t->cB = calloc((size_t)N_B * N_L * R1, 8);
    t->cT = calloc((size_t)N_T * R1, 8);   t->cS = calloc((size_t)N_S * R1, 8);
    if (!t->sR || !t->kR || !t->cR || !t->sU || !t->kU || !t->cU || !t->sN || !t->kN ||
        !t->cN || !t->sB || !t->cB || !t->cT || !t->cS) { or_tables_free(t); return 2; }
    const double Zd = (double)Z;
    const double lLmin = log(L_MIN), lLmax = log(L_MAX);

    /* relativistic segments: rows (g, L) */
    #pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < (N_R + N_U) * N_L; r++) {
        int seg_u = r >= N_R * N_L;
        int rr = seg_u ? r - N_R * N_L : r;
        int i = rr / N_L, l = rr % N_L;
        rowctx c; memset(&c, 0, sizeof c);
        c.kind = 0; c.Z = Zd;
        double u = seg_u ? axis_node(log(100.0), log(GMAX), N_U, i)
                         : axis_node(log(2.0), log(100.0), N_R, i);
        c.g1 = exp(u); c.g1m1 = c.g1 - 1.0;
        c.L = exp(axis_node(lLmin, lLmax, N_L, l));
        c.fc = seg_u ? t->fc : 0.0;
        c.Y = brems_yrange(c.g1, c.g1m1);
        double* S = seg_u ? t->sU : t->sR;
        double* K = seg_u ? t->kU : t->kR;
        double* CD = seg_u ? t->cU : t->cR;
        build_row(&c, 0, &S[rr], &K[rr], &CD[(size_t)rr * R1]);
    }
    /* non-relativistic segment: rows (g, eta_D, L_D) */
    #pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < N_NR * N_ETA * N_L; r++) {
        int i = r / (N_ETA * N_L), e = (r / N_L) % N_ETA, l = r % N_L;
        rowctx c; memset(&c, 0, sizeof c);
        c.kind = 1; c.Z = Zd;
        c.g1m1 = exp(axis_node(log(T_MIN_EV / MEC2EV), 0.0, N_NR, i));
        c.g1 = 1.0 + c.g1m1;
        c.ed = (double)e / (N_ETA - 1); c.etf = 1.0 - c.ed;
        c.Ltf = t->Ltf; c.Ld = exp(axis_node(lLmin, lLmax, N_L, l));
        c.Y = brems_yrange(c.g1, c.g1m1);
        build_row(&c, 0, &t->sN[r], &t->kN[r], &t->cN[(size_t)r * R1]);
    }
    /* Bethe-Heitler: rows (k, L) */
    #pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < N_B * N_L; r++) {
        int i = r / N_L, l = r % N_L;
        rowctx c; memset(&c, 0, sizeof c);
        c.kind = 2; c.Z = Zd;
        c.k = 2.0 + exp(axis_node(log(BH_X0), log(GMAX - 2.0), N_B, i));
        c.L = exp(axis_node(lLmin, lLmax, N_L, l));
        c.V = log(0.5 * c.k);
        build_row(&c, 1, &t->sB[r], NULL, &t->cB[(size_t)r * R1]);
    }
    /* Trident pair energy: rows g1 */
    for (int i = 0; i < N_T; i++) {
        rowctx c; memset(&c, 0, sizeof c);
        c.kind = 3; c.Z = Zd;
        c.g1 = exp(axis_node(log(3.0), log(GMAX), N_T, i));
        c.V = log(c.g1 - 1.0) - log(2.0);
        if (c.V > 0.0) build_row(&c, 0, NULL, NULL, &t->cT[(size_t)i * R1]);
        else for (int j = 0; j <= M_CDF; j++) t->cT[(size_t)i * R1 + j] = (double)j / M_CDF;
    }
    /* Trident positron split: rows g_pair */
    for (int i = 0; i < N_S; i++) {
        rowctx c; memset(&c, 0, sizeof c);
        c.kind = 4; c.Z = Zd;
        double gpair = exp(axis_node(log(4.0), log(GMAX), N_S, i));
        double q = 1.0 - 4.0 / gpair;
        double glo = 2.0 / (1.0 + sqrt(q > 0.0 ? q : 0.0));
        c.k = gpair; c.L = glo; c.V = log(gpair / (2.0 * glo));
        if (c.V > 0.0) build_row(&c, 1, NULL, NULL, &t->cS[(size_t)i * R1]);
        else for (int j = 0; j <= M_CDF; j++) t->cS[(size_t)i * R1 + j] = (double)j / M_CDF;
    }
    *out = t;
    return 0;
}

void or_tables_free(or_tables* t)
{
    if (!t) return;
    free(t->sR); free(t->kR); free(t->cR); free(t->sU); free(t->kU); free(t->cU);
    free(t->sN); free(t->kN); free(t->cN); free(t->sB); free(t->cB); free(t->cT); free(t->cS);
    free(t);
}

static const double* table_ptr(const or_tables* t, int which, int64_t* n)
{
    const int64_t R1 = M_CDF + 1;
    switch (which) {
    case 0:  *n = (int64_t)N_R * N_L; return t->sR;
    case 1:  *n = (int64_t)N_R * N_L; return t->kR;
    case 2:  *n = (int64_t)N_R * N_L * R1; return t->cR;
    case 3:  *n = (int64_t)N_U * N_L; return t->sU;
    case 4:  *n = (int64_t)N_U * N_L; return t->kU;
    case 5:  *n = (int64_t)N_U * N_L * R1; return t->cU;
    case 6:  *n = (int64_t)N_NR * N_ETA * N_L; return t->sN;
    case 7:  *n = (int64_t)N_NR * N_ETA * N_L; return t->kN;
    case 8:  *n = (int64_t)N_NR * N_ETA * N_L * R1; return t->cN;
    case 9:  *n = (int64_t)N_B * N_L; return t->sB;
    case 10: *n = (int64_t)N_B * N_L * R1; return t->cB;
    case 11: *n = (int64_t)N_T * R1; return t->cT;
    case 12: *n = (int64_t)N_S * R1; return t->cS;
    default: *n = 0; return NULL;
    }
}

int64_t or_tables_size(const or_tables* t, int which)
{
    int64_t n; table_ptr(t, which, &n); return n;
}

int or_tables_export(const or_tables* t, int which, double* dst, int64_t n)
{
    int64_t m; const double* p = table_ptr(t, which, &m);
    if (!p || n != m) return 1;
    memcpy(dst, p, (size_t)m * 8);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Table lookups: linear interpolation, first along the screening     */
/* axis (or axes), then along the energy axis.                        */
/* ------------------------------------------------------------------ */
static void axis_pos(double u, double u0, double u1, int n, int* i, double* w, int* inside)
{
    double du = (u1 - u0) / (n - 1);
    double pos = (u - u0) / du;
    if (pos <= 0.0) { *i = 0; *w = 0.0; *inside = 0; return; }
    if (pos >= n - 1) { *i = n - 2; *w = 1.0; *inside = 0; return; }
    int k = (int)pos;
    if (k > n - 2) k = n - 2;
    *i = k; *w = pos - k; *inside = 1;
}

static double lerp(double a, double b, double w) { return a + w * (b - a); }

typedef struct {
    double Z, Zs, ni, T;
    double scr[8];
    int iL, iE, iD; double wL, wE, wD; int inL, inE, inD;
    double lnLr, lnLd;
} cellstate;

static void cell_init(const or_tables* tb, double Zs, double ni, double T, cellstate* s)
{
    s->Z = tb->Z; s->Zs = Zs; s->ni = ni; s->T = T;
    or_screening(tb->Z, Zs, ni, T, s->scr);
    s->lnLr = log(s->scr[5]);
    axis_pos(s->lnLr, log(L_MIN), log(L_MAX), N_L, &s->iL, &s->wL, &s->inL);
    axis_pos(s->scr[3], 0.0, 1.0, N_ETA, &s->iE, &s->wE, &s->inE);
    s->lnLd = s->scr[3] > 0.0 ? log(s->scr[1]) : log(L_MIN);
    axis_pos(s->lnLd, log(L_MIN), log(L_MAX), N_L, &s->iD, &s->wD, &s->inD);
}

/* blend of a (g, L) table row-set at g-node i along L */
static double blendL(const double* T, int stride, int i, const cellstate* s, int col)
{
    const double* a = T + ((size_t)i * N_L + s->iL) * stride + col;
    return lerp(a[0], a[stride], s->wL);
}

/* blend of a (g, eta, L) table at g-node i: along L_D then eta_D */
static double blendN(const double* T, int stride, int i, const cellstate* s, int col)
{
    const double* a = T + (((size_t)i * N_ETA + s->iE) * N_L + s->iD) * stride + col;
    const double* b = a + (size_t)N_L * stride;
    double v0 = lerp(a[0], a[stride], s->wD);
    double v1 = lerp(b[0], b[stride], s->wD);
    return lerp(v0, v1, s->wE);
}

/* Bremsstrahlung segment of an electron of Lorentz factor g (g1m1 = g - 1) */
enum { SEG_NONE = 0, SEG_NR, SEG_R, SEG_U };
static int brems_segment(double g, double g1m1, double* u, int* high)
{
    *high = 0;
    if (!(g1m1 > T_MIN_EV / MEC2EV)) return SEG_NONE;
    if (g <= 2.0) { *u = log(g1m1); return SEG_NR; }
    if (g <= 100.0) { *u = log(g); return SEG_R; }
    if (g > GMAX) { *high = 1; *u = log(GMAX); return SEG_U; }
    *u = log(g);
    return SEG_U;
}

typedef struct {
    int seg, ig; double wg; int ing;
    double sig, sk;          /* sigma_B and its k-moment              */
    double dsig_du, dsk_du;  /* along the energy axis variable u       */
    double dsig_a, dsk_a;    /* along ln L_R (R/U) or ln L_D (NR)      */
    double dsig_e, dsk_e;    /* along eta_D (NR only)                  */
} brems_lookup_t;

static void brems_lookup(const or_tables* tb, const cellstate* s, double g, double g1m1,
                         brems_lookup_t* o, int* high)
{
    memset(o, 0, sizeof *o);
    double u;
    o->seg = brems_segment(g, g1m1, &u, high);
    if (o->seg == SEG_NONE) return;
    const int ax_n[4] = {0, N_NR, N_R, N_U};
    const double ax0[4] = {0, log(T_MIN_EV / MEC2EV), log(2.0), log(100.0)};
    const double ax1[4] = {0, 0.0, log(100.0), log(GMAX)};
    int n = ax_n[o->seg];
    axis_pos(u, ax0[o->seg], ax1[o->seg], n, &o->ig, &o->wg, &o->ing);
    double du = (ax1[o->seg] - ax0[o->seg]) / (n - 1);
    double S0, S1, K0, K1, dS0 = 0, dS1 = 0, dK0 = 0, dK1 = 0, eS0 = 0, eS1 = 0, eK0 = 0, eK1 = 0;
    if (o->seg == SEG_NR) {
        S0 = blendN(tb->sN, 1, o->ig, s, 0); S1 = blendN(tb->sN, 1, o->ig + 1, s, 0);
        K0 = blendN(tb->kN, 1, o->ig, s, 0); K1 = blendN(tb->kN, 1, o->ig + 1, s, 0);
        /* slopes of the bilinear screening blend */
        const double dLn = (log(L_MAX) - log(L_MIN)) / (N_L - 1), dEn = 1.0 / (N_ETA - 1);
        for (int q = 0; q < 2; q++) {
            const double* TS = q ? tb->kN : tb->sN;
            double sl[2], se[2];
            for (int h = 0; h < 2; h++) {
                const double* a = TS + ((size_t)(o->ig + h) * N_ETA + s->iE) * N_L + s->iD;
                const double* b = a + N_L;
                double v0 = lerp(a[0], a[1], s->wD), v1 = lerp(b[0], b[1], s->wD);
                sl[h] = s->inD ? lerp(a[1] - a[0], b[1] - b[0], s->wE) / dLn : 0.0;
                se[h] = s->inE ? (v1 - v0) / dEn : 0.0;
            }
            if (q) { dK0 = sl[0]; dK1 = sl[1]; eK0 = se[0]; eK1 = se[1]; }
            else   { dS0 = sl[0]; dS1 = sl[1]; eS0 = se[0]; eS1 = se[1]; }
        }
    } else {
        const double* TS = o->seg == SEG_R ? tb->sR : tb->sU;
        const double* TK = o->seg == SEG_R ? tb->kR : tb->kU;
        S0 = blendL(TS, 1, o->ig, s, 0); S1 = blendL(TS, 1, o->ig + 1, s, 0);
        K0 = blendL(TK, 1, o->ig, s, 0); K1 = blendL(TK, 1, o->ig + 1, s, 0);
        const double dLn = (log(L_MAX) - log(L_MIN)) / (N_L - 1);
        const double* a;
        a = TS + (size_t)o->ig * N_L + s->iL;       dS0 = s->inL ? (a[1] - a[0]) / dLn : 0.0;
        a = TS + (size_t)(o->ig + 1) * N_L + s->iL; dS1 = s->inL ? (a[1] - a[0]) / dLn : 0.0;
        a = TK + (size_t)o->ig * N_L + s->iL;       dK0 = s->inL ? (a[1] - a[0]) / dLn : 0.0;
        a = TK + (size_t)(o->ig + 1) * N_L + s->iL; dK1 = s->inL ? (a[1] - a[0]) / dLn : 0.0;
    }
    o->sig = lerp(S0, S1, o->wg);
    o->sk = lerp(K0, K1, o->wg);
    o->dsig_du = o->ing ? (S1 - S0) / du : 0.0;
    o->dsk_du = o->ing ? (K1 - K0) / du : 0.0;
    o->dsig_a = lerp(dS0, dS1, o->wg);
    o->dsk_a = lerp(dK0, dK1, o->wg);
    o->dsig_e = lerp(eS0, eS1, o->wg);
    o->dsk_e = lerp(eK0, eK1, o->wg);
}

static double bh_sigma(const or_tables* tb, const cellstate* s, double k, int* high, int* ik, double* wk)
{
    *high = 0;
    if (!(k > 2.0)) return 0.0;
    double km2 = k - 2.0;
    if (k > GMAX) { *high = 1; km2 = GMAX - 2.0; }
    int in;
    if (km2 < BH_X0) {
        /* below the first node: linear to zero at threshold (reading) */
        *ik = 0; *wk = 0.0;
        return blendL(tb->sB, 1, 0, s, 0) * (km2 / BH_X0);
    }
    axis_pos(log(km2), log(BH_X0), log(GMAX - 2.0), N_B, ik, wk, &in);
    double S0 = blendL(tb->sB, 1, *ik, s, 0), S1 = blendL(tb->sB, 1, *ik + 1, s, 0);
    return lerp(S0, S1, *wk);
}

/* inverse of the piecewise-linear blended CDF F(j), j = 0..M */
typedef struct { const double* T; int kind; int i; double w; const cellstate* s; } cdfsel;

static double cdf_at(const cdfsel* c, int j)
{
    const int R1 = M_CDF + 1;
    double a, b;
    switch (c->kind) {
    case 0: /* (g, L) */
        a = blendL(c->T, R1, c->i, c->s, j);
        b = blendL(c->T, R1, c->i + 1, c->s, j);
        return lerp(a, b, c->w);
    case 1: /* NR (g, eta, L) */
        a = blendN(c->T, R1, c->i, c->s, j);
        b = blendN(c->T, R1, c->i + 1, c->s, j);
        return lerp(a, b, c->w);
    default: /* 1-D row set */
        a = c->T[(size_t)c->i * R1 + j];
        b = c->T[(size_t)(c->i + 1) * R1 + j];
        return lerp(a, b, c->w);
    }
}

/* Returns t and, in *ct, 1 - t evaluated from F_hi - xi, which keeps its
 * relative precision near the top of the row (the spectrum tip, where the
 * product's gamma - 1 is small). */
static double cdf_invert(const cdfsel* c, double xi, double* ct)
{
    int lo = 0, hi = M_CDF;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (cdf_at(c, mid) <= xi) lo = mid; else hi = mid;
    }
    double Flo = cdf_at(c, lo), Fhi = cdf_at(c, hi), d = Fhi - Flo;
    *ct = ((M_CDF - hi) + (Fhi - xi) / d) / M_CDF;
    return (lo + (xi - Flo) / d) / M_CDF;
}

/* Bremsstrahlung photon energy, Sec. III.A: t from the blended CDF, then
 * k from the row abscissa of the actual g1.  Returns k, g2, g2 - 1. */
static void brems_sample(const or_tables* tb, const cellstate* s, const brems_lookup_t* L,
                         double g1, double g1m1, double xi, double* k, double* g2, double* g2m1)
{
    cdfsel c;
    c.s = s; c.i = L->ig; c.w = L->wg;
    if (L->seg == SEG_NR) { c.T = tb->cN; c.kind = 1; }
    else { c.T = L->seg == SEG_R ? tb->cR : tb->cU; c.kind = 0; }
    double ct;
    cdf_invert(&c, xi, &ct);
    double Y = brems_yrange(g1, g1m1);
    double dl = L->seg == SEG_NR ? ct * ct * Y : ct * Y;
    brems_kin(g1, g1m1, dl, k, g2, g2m1);
}

static void bh_sample(const or_tables* tb, const cellstate* s, double k, int ik, double wk,
                      double xi, double* gp, double* gm)
{
    cdfsel c; c.T = tb->cB; c.kind = 0; c.i = ik; c.w = wk; c.s = s;
    double ct, t = cdf_invert(&c, xi, &ct);
    double V = log(0.5 * k);
    if (t <= 0.5) { *gp = exp(2.0 * t * V); *gm = k - *gp; }
    else          { *gm = exp(2.0 * ct * V); *gp = k - *gm; }
}

/* Trident: pair energy on [2, g1 - 1] in ln g_pair, then the positron
 * split; *gfm1 = g1 - 1 - g_pair, the electron's kinetic energy left,
 * from the complement of the abscissa (no cancellation at the tip). */
static void trident_sample(const or_tables* tb, double g1, double g1m1, double xi1, double xi2,
                           double* gpair, double* gp, double* gm, double* gfm1)
{
    cdfsel c; c.s = NULL; c.kind = 2;
    int in;
    double ga = g1 > GMAX ? GMAX : g1;
    c.T = tb->cT;
    axis_pos(log(ga), log(3.0), log(GMAX), N_T, &c.i, &c.w, &in);
    double ct, t = cdf_invert(&c, xi1, &ct);
    double Lg = log(g1m1) - log(2.0);
    *gpair = exp(log(2.0) + t * Lg);
    *gfm1 = -g1m1 * expm1(-ct * Lg);
    if (*gpair <= 4.0) { *gp = 0.5 * (*gpair); *gm = *gp; return; }
    double gq = *gpair > GMAX ? GMAX : *gpair;
    c.T = tb->cS;
    axis_pos(log(gq), log(4.0), log(GMAX), N_S, &c.i, &c.w, &in);
    double ct2, t2 = cdf_invert(&c, xi2, &ct2);
    double q = 1.0 - 4.0 / (*gpair);
    double glo = 2.0 / (1.0 + sqrt(q));
    double V = log(*gpair / (2.0 * glo));
    if (t2 <= 0.5) { *gp = glo * exp(2.0 * t2 * V); *gm = *gpair - *gp; }
    else           { *gm = glo * exp(2.0 * ct2 * V); *gp = *gpair - *gm; }
}

/* process ids of or_lookup / or_sample: 1 Brems, 2 BH, 4 Trident */
int or_lookup(const or_tables* t, double Zs, double ni, double T, double e1, int process, double out[4])
{
    cellstate s; cell_init(t, Zs, ni, T, &s);
    int high = 0;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (process == OR_BREMS) {
        brems_lookup_t L;
        double p2 = e1 * e1 - 1.0;
        brems_lookup(t, &s, e1, p2 / (e1 + 1.0), &L, &high);
        out[0] = L.sig; out[1] = L.sk; out[2] = L.seg; out[3] = high;
    } else if (process == OR_BH) {
        int ik; double wk;
        out[0] = bh_sigma(t, &s, e1, &high, &ik, &wk); out[3] = high;
    } else if (process == OR_TRIDENT) {
        out[0] = or_sigma_trident(t->Z, e1);
    } else return 1;
    return 0;
}

int or_sample(const or_tables* t, double Zs, double ni, double T, double e1, int process,
              double xi1, double xi2, double out[2])
{
    cellstate s; cell_init(t, Zs, ni, T, &s);
    int high = 0;
    if (process == OR_BREMS) {
        brems_lookup_t L;
        double g1m1 = (e1 * e1 - 1.0) / (e1 + 1.0);
        brems_lookup(t, &s, e1, g1m1, &L, &high);
        if (L.seg == SEG_NONE) return 1;
        double k, g2, g2m1;
        brems_sample(t, &s, &L, e1, g1m1, xi1, &k, &g2, &g2m1);
        out[0] = k; out[1] = g2;
    } else if (process == OR_BH) {
        int ik = 0; double wk = 0.0;
        if (bh_sigma(t, &s, e1, &high, &ik, &wk) <= 0.0) return 1;
        bh_sample(t, &s, e1, ik, wk, xi1, &out[0], &out[1]);
    } else if (process == OR_TRIDENT) {
        if (!(e1 > 3.0)) return 1;
        double gpair, gp, gm, gfm1;
        trident_sample(t, e1, (e1 * e1 - 1.0) / (e1 + 1.0), xi1, xi2, &gpair, &gp, &gm, &gfm1);
        out[0] = gp; out[1] = gm;
    } else return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and U(0,1) with   */
/* 53 random bits                                                      */
/* ------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)m1;
        uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)m0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double or_u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* counter layout: (x, cell, step low word, tag<<24 | step bits 32..55) */
static void draw(uint64_t seed, uint64_t step, uint32_t cell, uint32_t x, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = { x, cell, (uint32_t)step, (tag << 24) | ((uint32_t)(step >> 32) & 0xFFFFFFu) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    or_philox(ctr, key, out);
}

enum { TAG_KEY_E = 0x01, TAG_KEY_IE = 0x02, TAG_KEY_G = 0x03, TAG_KEY_IG = 0x04,
       TAG_ACC_BR = 0x11, TAG_SMP_BR = 0x12, TAG_HI_BR = 0x13,
       TAG_ACC_TR = 0x21, TAG_SMP_TR = 0x22, TAG_HI_TR = 0x23,
       TAG_ACC_BH = 0x31, TAG_SMP_BH = 0x32, TAG_HI_BH = 0x33 };

/* The two uniforms of a pair's acceptance test, eq:proba3 (U1 against P,  */
/* U2 against W_ion/max(W_mobile, W_ion)), for the pair whose numbers are  */
/* keyed by x.  Reading (the paper fixes no generator): U1 has 53 random   */
/* bits, the upper 32 of them word ((x >> 8) & 3) of the draw with the    */
/* process's "hi" tag keyed by ((x >> 10) << 8) | (x & 255), so that four */
/* pairs share one draw, the lower 21 the top bits of word 0 of the       */
/* pair's own draw with the acceptance tag; U2 is u53 of words 2 and 3 of */
/* that draw.                                                              */
void or_accept_uniforms(uint64_t seed, uint64_t step, uint32_t cell, uint32_t x, uint32_t tag,
                        uint32_t tag_hi, double* U1, double* U2)
{
    uint32_t h[4], r[4];
    draw(seed, step, cell, ((x >> 10) << 8) | (x & 255u), tag_hi, h);
    draw(seed, step, cell, x, tag, r);
    *U1 = ((double)h[(x >> 8) & 3u] * 2097152.0 + (double)(r[0] >> 11)) * (1.0 / 9007199254740992.0);
    *U2 = or_u53(r[2], r[3]);
}

/* ------------------------------------------------------------------ */
/* Pairing, Sec. III.A: N = max(N_a, N_b) macro-pairs, each drawn     */
/* uniformly.  Reading: each species is ordered by a 32-bit Philox key */
/* per particle (ties by index); the larger species A is walked once   */
/* in that order and the smaller one B cyclically, pair j =            */
/* (A[pi_A(j)], B[pi_B(j mod N_B)]); a tie N_a = N_b makes the mobile  */
/* species A.  The random numbers of pair j are keyed by              */
/* x = i + k N_m: i is the index of its mobile particle and k = j div  */
/* N_m counts that particle's earlier pairs in the pass (k = 0 when    */
/* every mobile particle pairs once).  Every pair of a pass has its    */
/* own counter, and the key does not depend on the order of the pairs. */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t key; int32_t idx; } keyidx;

static int cmp_keyidx(const void* x, const void* y)
{
    const keyidx* a = (const keyidx*)x; const keyidx* b = (const keyidx*)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx);
}

static void key_order(int32_t n, uint64_t seed, uint64_t step, uint32_t cell, uint32_t tag,
                      int32_t* order, keyidx* scratch)
{
    uint32_t r[4];
    for (int32_t i = 0; i < n; i++) {
        if ((i & 3) == 0) draw(seed, step, cell, (uint32_t)i >> 2, tag, r);
        scratch[i].key = r[i & 3];
        scratch[i].idx = i;
    }
    qsort(scratch, (size_t)n, sizeof(keyidx), cmp_keyidx);
    for (int32_t i = 0; i < n; i++) order[i] = scratch[i].idx;
}

/* fills pa[j], pb[j] (local indices of the a and b particle of pair j) */
static int64_t pair_one_cell(int32_t na, int32_t nb, uint64_t seed, uint64_t step, uint32_t cell,
                             uint32_t tag_a, uint32_t tag_b, int32_t* pa, int32_t* pb)
{
    if (na <= 0 || nb <= 0) return 0;
    int32_t n = na > nb ? na : nb;
    int32_t* oa = (int32_t*)malloc(sizeof(int32_t) * (size_t)(na + nb));
    keyidx* sc = (keyidx*)malloc(sizeof(keyidx) * (size_t)n);
    int32_t* ob = oa + na;
    key_order(na, seed, step, cell, tag_a, oa, sc);
    key_order(nb, seed, step, cell, tag_b, ob, sc);
    for (int32_t j = 0; j < n; j++) {
        if (na >= nb) { pa[j] = oa[j]; pb[j] = ob[j % nb]; }
        else          { pb[j] = ob[j]; pa[j] = oa[j % na]; }
    }
    free(oa); free(sc);
    return n;
}

int or_pair_cells(int64_t n_cells, const int64_t* cell_id, const int64_t* a_off, const int32_t* a_cnt,
                  const int64_t* b_off, const int32_t* b_cnt,
                  const double* wa, const double* wb,
                  uint64_t seed, uint64_t step, uint32_t pass,
                  const int64_t* pair_off, int32_t* pa, int32_t* pb, double* n_ab)
{
    uint32_t ta = pass == 1 ? TAG_KEY_E : TAG_KEY_G;
    uint32_t tb = pass == 1 ? TAG_KEY_IE : TAG_KEY_IG;
    if (pass != 1 && pass != 2) return 1;
    for (int64_t c = 0; c < n_cells; c++) {
        int32_t na = a_cnt ? a_cnt[c] : (int32_t)(a_off[c + 1] - a_off[c]);
        int32_t nb = b_cnt ? b_cnt[c] : (int32_t)(b_off[c + 1] - b_off[c]);
        uint32_t cell = (uint32_t)(cell_id ? cell_id[c] : c);
        int64_t n = pair_one_cell(na, nb, seed, step, cell, ta, tb,
                                  pa + pair_off[c], pb + pair_off[c]);
        if (n_ab) {
            double s = 0.0;
            for (int64_t j = 0; j < n; j++) {
                double x = wa[a_off[c] + pa[pair_off[c] + j]], y = wb[b_off[c] + pb[pair_off[c] + j]];
                s += x < y ? x : y;
            }
            n_ab[c] = s;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Lorentz transforms to / from the ion rest frame, Sec. III.A.        */
/* Reading: the boost is along the ion velocity (the printed last      */
/* factor beta_e is read as beta_i).  u is the ion's proper velocity   */
/* gamma_i beta_i; (E, p) -> (E', p') with                             */
/*   E' = g_i E - u.p,  p' = p + [u.p/(g_i + 1) - E] u.                */
/* ------------------------------------------------------------------ */
static void to_ion(const double u[3], double gi, double E, const double p[3], double* Ep, double pp[3])
{
    double up = u[0] * p[0] + u[1] * p[1] + u[2] * p[2];
    double f = up / (gi + 1.0) - E;
    *Ep = gi * E - up;
    for (int d = 0; d < 3; d++) pp[d] = p[d] + f * u[d];
}

static void from_ion(const double u[3], double gi, double Ep, const double pp[3], double p[3])
{
    double up = u[0] * pp[0] + u[1] * pp[1] + u[2] * pp[2];
    double f = up / (gi + 1.0) + Ep;
    for (int d = 0; d < 3; d++) p[d] = pp[d] + f * u[d];
}

/* The same two transforms for one 4-vector, exported for the pins:
 * out = (E', p'x, p'y, p'z) in the ion rest frame, and back (momentum). */
void or_to_ion(const double u[3], double E, const double p[3], double out[4])
{
    double gi = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    to_ion(u, gi, E, p, &out[0], out + 1);
}

void or_from_ion(const double u[3], double Ep, const double pp[3], double out[3])
{
    double gi = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    from_ion(u, gi, Ep, pp, out);
}

/* ------------------------------------------------------------------ */
/* The Monte Carlo step, Sec. III.A, one cell, sequential in j.        */
/* ------------------------------------------------------------------ */
typedef struct {
    const or_tables* tb;
    or_species *el, *ph, *nel, *npo;
    const or_species* ion;
    double dt; uint64_t seed, step; uint32_t proc; double near_rel;
} stepctx;

static int append(or_species* sl, int64_t c, double px, double py, double pz, double w, int64_t parent)
{
    int64_t cap = sl->off[c + 1] - sl->off[c];
    if (sl->count[c] >= cap) return 0;
    int64_t at = sl->off[c] + sl->count[c];
    sl->px[at] = px; sl->py[at] = py; sl->pz[at] = pz; sl->w[at] = w;
    if (sl->parent) sl->parent[at] = parent;
    sl->count[c]++;
    return 1;
}

/* Lab-frame energy change of the electron, from its ion-frame change
 * dE' (= -k or -g_pair, exact by construction) rather than from the
 * difference of two Lorentz factors, which cancels when dE' << gamma:
 * dE_lab = g_i dE' + u.n (|p'_f| - |p'|), |p'_f| - |p'| = dE'(g'_f + g')/(|p'_f| + |p'|). */
static double lab_energy_change(int moving, const double u[3], double gi, const double n[3],
                                double dEp, double gfp, double gp, double pf, double pm)
{
    if (!moving) return dEp;
    double dp = dEp * (gfp + gp) / (pf + pm);
    return gi * dEp + (u[0] * n[0] + u[1] * n[1] + u[2] * n[2]) * dp;
}

static int32_t cell_step(const stepctx* X, const or_cells* cells, int64_t c, int64_t* ti, double* td)
{
    const or_tables* tb = X->tb;
    int32_t st = 0;
    double Zs = cells->Zstar[c], ni = cells->n_i[c], T = cells->T_e[c];
    if (!(Zs >= 0.0 && Zs <= tb->Z && ni > 0.0 && T >= 0.0 && isfinite(ni) && isfinite(T)))
        return OR_ST_BAD_CELL;
    or_species* el = X->el; or_species* ph = X->ph; const or_species* io = X->ion;
    int64_t e0 = el->off[c], g0 = ph->off[c], i0 = io->off[c];
    int32_t Ne = el->count ? el->count[c] : (int32_t)(el->off[c + 1] - e0);
    int32_t Ng = ph->count ? ph->count[c] : (int32_t)(ph->off[c + 1] - g0);
    int32_t Ni = io->count ? io->count[c] : (int32_t)(io->off[c + 1] - i0);
    double ne = 0.0, ng = 0.0, nI = 0.0;
    for (int32_t a = 0; a < Ne; a++) ne += el->w[e0 + a];
    for (int32_t a = 0; a < Ng; a++) ng += ph->w[g0 + a];
    for (int32_t a = 0; a < Ni; a++) nI += io->w[i0 + a];
    int badw = !(isfinite(ne) && isfinite(ng) && isfinite(nI));
    for (int32_t a = 0; a < Ne && !badw; a++) badw |= !(el->w[e0 + a] >= 0.0);
    for (int32_t a = 0; a < Ng && !badw; a++) badw |= !(ph->w[g0 + a] >= 0.0);
    for (int32_t a = 0; a < Ni && !badw; a++) badw |= !(io->w[i0 + a] >= 0.0);
    if (badw) return OR_ST_BAD_WEIGHT;

    cellstate s;
    cell_init(tb, Zs, ni, T, &s);
    const int moving = io->px != NULL;
    int32_t nmax = Ne > Ni ? Ne : Ni;
    if (Ng > nmax) nmax = Ng;
    int32_t* pa = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * nmax + 2));
    int32_t* pb = pa + nmax + 1;
    uint32_t cell = (uint32_t)(cells->cell_id ? cells->cell_id[c] : c);

    /* ---- electron-ion pass: Bremsstrahlung then Trident per pair ---- */
    if ((X->proc & (OR_BREMS | OR_TRIDENT)) && Ne > 0 && Ni > 0) {
        int64_t N = pair_one_cell(Ne, Ni, X->seed, X->step, cell, TAG_KEY_E, TAG_KEY_IE, pa, pb);
        double nab = 0.0;
        for (int64_t j = 0; j < N; j++) {
            double x = el->w[e0 + pa[j]], y = io->w[i0 + pb[j]];
            nab += x < y ? x : y;
        }
        td[OR_D_NAB_EI] = nab;
        double coef = ne * nI / nab;
        if (!(nab > 0.0)) N = 0;
        for (int64_t j = 0; j < N; j++) {
            int64_t ie = e0 + pa[j], ii = i0 + pb[j];
            /* the pair's random numbers: keyed by its electron when every
             * electron pairs once (N_e >= N_i), else by the pair index */
            uint32_t dkey = (uint32_t)(pa[j] + (j / Ne) * Ne);
            double We = el->w[ie], Wi = io->w[ii];
            double Pej = Wi / (We > Wi ? We : Wi);
            double u[3] = {0, 0, 0}, gi = 1.0;
            if (moving) {
                u[0] = io->px[ii]; u[1] = io->py[ii]; u[2] = io->pz[ii];
                gi = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            }
            for (int proc = 0; proc < 2; proc++) {
                uint32_t pbit = proc == 0 ? OR_BREMS : OR_TRIDENT;
                if (!(X->proc & pbit)) continue;
                ti[proc == 0 ? OR_I_PAIRS_BR : OR_I_PAIRS_TR]++;
                double p[3] = { el->px[ie], el->py[ie], el->pz[ie] };
                double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
                double ge = sqrt(1.0 + p2);
                double gpm1, pp[3], gp;   /* ion-frame gamma - 1, momentum, gamma */
                if (moving) {
                    to_ion(u, gi, ge, p, &gp, pp);
                    double q2 = pp[0] * pp[0] + pp[1] * pp[1] + pp[2] * pp[2];
                    gpm1 = q2 / (sqrt(1.0 + q2) + 1.0);
                } else {
                    pp[0] = p[0]; pp[1] = p[1]; pp[2] = p[2];
                    gp = ge; gpm1 = p2 / (ge + 1.0);
                }
                double pm = sqrt(pp[0] * pp[0] + pp[1] * pp[1] + pp[2] * pp[2]);
                double sig; int high = 0;
                brems_lookup_t BL;
                if (proc == 0) { brems_lookup(tb, &s, gp, gpm1, &BL, &high); sig = BL.sig; }
                else sig = or_sigma_trident(tb->Z, gp);
                if (high) st |= OR_ST_GAMMA_HIGH;
                if (!(sig > 0.0)) continue;
                /* eq:proba3 with the invariant of eq:proba2: g' v' = c |p'| */
                double x = coef * sig * (CLIGHT * pm / (ge * gi)) * X->dt;
                double P = -expm1(-x);
                uint32_t r[4];
                double U1, U2;
                or_accept_uniforms(X->seed, X->step, cell, dkey, proc == 0 ? TAG_ACC_BR : TAG_ACC_TR,
                                proc == 0 ? TAG_HI_BR : TAG_HI_TR, &U1, &U2);
                if (fabs(U1 - P) <= X->near_rel * P) ti[proc == 0 ? OR_I_NEAR_BR : OR_I_NEAR_TR]++;
                if (!(U1 < P && U2 < Pej)) continue;
                draw(X->seed, X->step, cell, dkey, proc == 0 ? TAG_SMP_BR : TAG_SMP_TR, r);
                double xi1 = or_u53(r[0], r[1]), xi2 = or_u53(r[2], r[3]);
                double sc = 1.0 / pm;
                double nh[3] = { pp[0] * sc, pp[1] * sc, pp[2] * sc };
                if (proc == 0) {
                    /* Sec. III.A: photon along the electron, g'_ef = g' - k' */
                    double k, g2, g2m1;
                    brems_sample(tb, &s, &BL, gp, gpm1, xi1, &k, &g2, &g2m1);
                    double pf = sqrt(g2m1 * (g2 + 1.0));
                    double qe[3], qk[3];
                    if (moving) {
                        double a[3] = { nh[0] * pf, nh[1] * pf, nh[2] * pf };
                        double b[3] = { nh[0] * k, nh[1] * k, nh[2] * k };
                        from_ion(u, gi, g2, a, qe);
                        from_ion(u, gi, k, b, qk);
                    } else {
                        double f = pf / pm, h = k / pm;
                        qe[0] = p[0] * f; qe[1] = p[1] * f; qe[2] = p[2] * f;
                        qk[0] = p[0] * h; qk[1] = p[1] * h; qk[2] = p[2] * h;
                    }
                    el->px[ie] = qe[0]; el->py[ie] = qe[1]; el->pz[ie] = qe[2];
                    double kl = sqrt(qk[0] * qk[0] + qk[1] * qk[1] + qk[2] * qk[2]);
                    ti[OR_I_EV_BR]++;
                    td[OR_D_E_BR] += We * kl;
                    td[OR_D_DE_EL] += We * lab_energy_change(moving, u, gi, nh, -k, g2, gp, pf, pm);
                    td[OR_D_W_BR] += We;
                    if (!append(ph, c, qk[0], qk[1], qk[2], We, ie)) { ti[OR_I_DROP_PH]++; st |= OR_ST_OVERFLOW; }
                } else {
                    /* Trident: pair energy, then the positron split; the pair
                     * travels along the electron, which loses g_pair (reading) */
                    double gpair, gpl, gmi, gfm1;
                    trident_sample(tb, gp, gpm1, xi1, xi2, &gpair, &gpl, &gmi, &gfm1);
                    double gf = gfm1 + 1.0;
                    double pf = sqrt(gfm1 * (gf + 1.0));
                    double pplus = sqrt((gpl - 1.0) * (gpl + 1.0)), pminus = sqrt((gmi - 1.0) * (gmi + 1.0));
                    double qe[3], qp[3], qm[3];
                    if (moving) {
                        double a[3] = { nh[0] * pf, nh[1] * pf, nh[2] * pf };
                        double b[3] = { nh[0] * pplus, nh[1] * pplus, nh[2] * pplus };
                        double d[3] = { nh[0] * pminus, nh[1] * pminus, nh[2] * pminus };
                        from_ion(u, gi, gf, a, qe);
                        from_ion(u, gi, gpl, b, qp);
                        from_ion(u, gi, gmi, d, qm);
                    } else {
                        double f = pf / pm, fp = pplus / pm, fm = pminus / pm;
                        for (int dd = 0; dd < 3; dd++) { qe[dd] = p[dd] * f; qp[dd] = p[dd] * fp; qm[dd] = p[dd] * fm; }
                    }
                    el->px[ie] = qe[0]; el->py[ie] = qe[1]; el->pz[ie] = qe[2];
                    double gpl_l = sqrt(1.0 + qp[0] * qp[0] + qp[1] * qp[1] + qp[2] * qp[2]);
                    double gmi_l = sqrt(1.0 + qm[0] * qm[0] + qm[1] * qm[1] + qm[2] * qm[2]);
                    ti[OR_I_EV_TR]++;
                    td[OR_D_E_TR] += We * (gpl_l + gmi_l);
                    td[OR_D_DE_EL] += We * lab_energy_change(moving, u, gi, nh, -gpair, gf, gp, pf, pm);
                    td[OR_D_W_TR] += We;
                    if (!append(X->nel, c, qm[0], qm[1], qm[2], We, ie)) { ti[OR_I_DROP_EL]++; st |= OR_ST_OVERFLOW; }
                    if (!append(X->npo, c, qp[0], qp[1], qp[2], We, ie)) { ti[OR_I_DROP_PO]++; st |= OR_ST_OVERFLOW; }
                }
            }
        }
    }

    /* ---- photon-ion pass: Bethe-Heitler over photons alive at step start ---- */
    if ((X->proc & OR_BH) && Ng > 0 && Ni > 0) {
        int64_t N = pair_one_cell(Ng, Ni, X->seed, X->step, cell, TAG_KEY_G, TAG_KEY_IG, pa, pb);
        unsigned char* dead = (unsigned char*)calloc((size_t)Ng, 1);
        double nab = 0.0;
        for (int64_t j = 0; j < N; j++) {
            double x = ph->w[g0 + pa[j]], y = io->w[i0 + pb[j]];
            nab += x < y ? x : y;
        }
        td[OR_D_NAB_GI] = nab;
        double coef = ng * nI / nab;
        int any_dead = 0;
        if (!(nab > 0.0)) N = 0;
        for (int64_t j = 0; j < N; j++) {
            if (dead[pa[j]]) continue;
            int64_t ig = g0 + pa[j], ii = i0 + pb[j];
            /* keyed by the photon when every photon pairs once, else by j */
            uint32_t dkey = (uint32_t)(pa[j] + (j / Ng) * Ng);
            ti[OR_I_PAIRS_BH]++;
            double Wg = ph->w[ig], Wi = io->w[ii];
            double Pej = Wi / (Wg > Wi ? Wg : Wi);
            double q[3] = { ph->px[ig], ph->py[ig], ph->pz[ig] };
            double k = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
            double u[3] = {0, 0, 0}, gi = 1.0, kp = k, qp[3] = { q[0], q[1], q[2] };
            if (moving) {
                u[0] = io->px[ii]; u[1] = io->py[ii]; u[2] = io->pz[ii];
                gi = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                to_ion(u, gi, k, q, &kp, qp);
            }
            int high = 0, ik = 0; double wk = 0.0;
            double sig = bh_sigma(tb, &s, kp, &high, &ik, &wk);
            if (high) st |= OR_ST_GAMMA_HIGH;
            if (!(sig > 0.0)) continue;
            /* eq:proba3 with sigma_BH, n_gamma, and the flux factor k' c/(k g_i) */
            double x = coef * sig * (CLIGHT * kp / (k * gi)) * X->dt;
            double P = -expm1(-x);
            uint32_t r[4];
            double U1, U2;
            or_accept_uniforms(X->seed, X->step, cell, dkey, TAG_ACC_BH, TAG_HI_BH, &U1, &U2);
            if (fabs(U1 - P) <= X->near_rel * P) ti[OR_I_NEAR_BH]++;
            if (!(U1 < P && U2 < Pej)) continue;
            draw(X->seed, X->step, cell, dkey, TAG_SMP_BH, r);
            double xi = or_u53(r[0], r[1]);
            double gpl, gmi;
            bh_sample(tb, &s, kp, ik, wk, xi, &gpl, &gmi);
            double pplus = sqrt((gpl - 1.0) * (gpl + 1.0)), pminus = sqrt((gmi - 1.0) * (gmi + 1.0));
            double qpl[3], qmi[3];
            if (moving) {
                double sc = 1.0 / kp;
                double a[3] = { qp[0] * sc * pplus, qp[1] * sc * pplus, qp[2] * sc * pplus };
                double b[3] = { qp[0] * sc * pminus, qp[1] * sc * pminus, qp[2] * sc * pminus };
                from_ion(u, gi, gpl, a, qpl);
                from_ion(u, gi, gmi, b, qmi);
            } else {
                double fp = pplus / k, fm = pminus / k;
                for (int d = 0; d < 3; d++) { qpl[d] = q[d] * fp; qmi[d] = q[d] * fm; }
            }
            double gpl_l = sqrt(1.0 + qpl[0] * qpl[0] + qpl[1] * qpl[1] + qpl[2] * qpl[2]);
            double gmi_l = sqrt(1.0 + qmi[0] * qmi[0] + qmi[1] * qmi[1] + qmi[2] * qmi[2]);
            dead[pa[j]] = 1; any_dead = 1;
            ti[OR_I_EV_BH]++;
            td[OR_D_E_BH] += Wg * (gpl_l + gmi_l);
            td[OR_D_DE_PH] += -Wg * k;
            td[OR_D_W_BH] += Wg;
            if (!append(X->nel, c, qmi[0], qmi[1], qmi[2], Wg, ig)) { ti[OR_I_DROP_EL]++; st |= OR_ST_OVERFLOW; }
            if (!append(X->npo, c, qpl[0], qpl[1], qpl[2], Wg, ig)) { ti[OR_I_DROP_PO]++; st |= OR_ST_OVERFLOW; }
        }
        /* end of step: stable removal of converted photons; the photons
         * created this step (after index Ng) follow the survivors */
        if (any_dead) {
            int32_t n = ph->count[c], wpos = 0;
            for (int32_t a = 0; a < n; a++) {
                if (a < Ng && dead[a]) continue;
                if (wpos != a) {
                    ph->px[g0 + wpos] = ph->px[g0 + a]; ph->py[g0 + wpos] = ph->py[g0 + a];
                    ph->pz[g0 + wpos] = ph->pz[g0 + a]; ph->w[g0 + wpos] = ph->w[g0 + a];
                    if (ph->parent) ph->parent[g0 + wpos] = ph->parent[g0 + a];
                }
                wpos++;
            }
            ph->count[c] = wpos;
        }
        free(dead);
    }
    free(pa);
    return st;
}

int or_collide_step(const or_tables* t, const or_cells* cells,
                    or_species* el, or_species* ph, const or_species* ion,
                    or_species* new_el, or_species* new_po,
                    double dt, uint64_t seed, uint64_t step, uint32_t processes,
                    double near_rel, int64_t* tal_i, double* tal_d, int32_t* status,
                    int nthreads)
{
    if (!t || !cells || !el || !ph || !ion || !new_el || !new_po || !tal_i || !tal_d) return 1;
    if (!ph->count || !new_el->count || !new_po->count) return 1;
    if (!(dt > 0.0)) return 1;
    stepctx X;
    X.tb = t; X.el = el; X.ph = ph; X.ion = ion; X.nel = new_el; X.npo = new_po;
    X.dt = dt; X.seed = seed; X.step = step; X.proc = processes; X.near_rel = near_rel;
    int32_t st = 0;
    int64_t n = cells->n_cells;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    memset(tal_i, 0, sizeof(int64_t) * (size_t)n * OR_NI);
    memset(tal_d, 0, sizeof(double) * (size_t)n * OR_ND);
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:st)
    for (int64_t c = 0; c < n; c++)
        st |= cell_step(&X, cells, c, tal_i + c * OR_NI, tal_d + c * OR_ND);
    if (status) *status |= st;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Expected yield: Y_c = sum_j w_j P_j <k>_j with P = 1 - exp(-x),    */
/* x = n_i sigma_B(g) beta c dt against the background ions of the     */
/* cell (eq:proba1), n_i = n_e/Z* (Sec. II.A), <k> = sigma_k/sigma_B.  */
/* ------------------------------------------------------------------ */
typedef struct {
    double dlnLr[3];   /* d ln L_R / d(Z*, n_e, T_e)      */
    double deta[3];    /* d eta_D / d(...)                */
    double dlnLd[3];   /* d ln L_D / d(...)               */
    double dlnni[3];   /* d ln n_i / d(...)               */
} cellgrad;

/* chain rule of the screening state (eq:LDH, eq:ITFD, eq:reduit) */
static void cell_jacobian(const cellstate* s, double ne, cellgrad* G)
{
    const double Zs = s->Zs, T = s->T, Z = s->Z;
    double Ltf = s->scr[0], Ld = s->scr[1], etf = s->scr[2], ed = s->scr[3];
    double br = s->scr[6];
    memset(G, 0, sizeof *G);
    G->dlnni[0] = -1.0 / Zs; G->dlnni[1] = 1.0 / ne; G->dlnni[2] = 0.0;
    G->deta[0] = 1.0 / Z;
    if (br == 1.0) {        /* L_D^2 = eps0 T / (e n_e (Zs+1)) */
        G->dlnLd[0] = -0.5 / (Zs + 1.0); G->dlnLd[1] = -0.5 / ne; G->dlnLd[2] = 0.5 / T;
    } else if (br == 2.0) { /* L_D = r_i = (3 Zs / (4 pi n_e))^(1/3) */
        G->dlnLd[0] = 1.0 / (3.0 * Zs); G->dlnLd[1] = -1.0 / (3.0 * ne); G->dlnLd[2] = 0.0;
    }
    /* a = I_TFD(etf, ed, Ltf, Ld) */
    double A = Ltf * Ltf, B = Ld * Ld, D = B - A, M = A > B ? A : B;
    double X = itfd_cross(Ltf, Ld), dXdB;
    if (fabs(D) <= 1e-4 * M) {
        double m = 0.5 * (A + B), h2 = log1p(m) - m / (1.0 + m), h2p = m / ((1.0 + m) * (1.0 + m));
        dXdB = A * h2 / (m * m) - A * B * h2 / (m * m * m) + A * B * h2p / (2.0 * m * m);
    } else {
        dXdB = A * (log1p(D / (1.0 + A)) - D / (1.0 + B)) / (D * D);
    }
    double da_ded = -etf * h_single(Ltf) + ed * h_single(Ld) + (etf - ed) * X;
    double da_dlnLd = ed * ed * B * B / ((1.0 + B) * (1.0 + B)) + etf * ed * 2.0 * B * dXdB;
    double x = s->scr[5] * s->scr[5];
    double dlnLr_da = ((x + 1.0) / x) * ((x + 1.0) / x);
    for (int q = 0; q < 3; q++)
        G->dlnLr[q] = dlnLr_da * (da_ded * G->deta[q] + da_dlnLd * G->dlnLd[q]);
}

static double yield_one(const or_tables* tb, const cellstate* s, double ni, double px, double py,
                        double pz, double w, double dt, double gout[3], double* gw, double gcell[3],
                        double gabs[3], const cellgrad* G, double gY)
{
    double p2 = px * px + py * py + pz * pz, g = sqrt(1.0 + p2), gm1 = p2 / (g + 1.0);
    brems_lookup_t L; int high;
    brems_lookup(tb, s, g, gm1, &L, &high);
    if (gout) { gout[0] = gout[1] = gout[2] = 0.0; }
    if (gw) *gw = 0.0;
    if (!(L.sig > 0.0)) return 0.0;
    double beta = sqrt(p2) / g;
    double x = ni * L.sig * beta * CLIGHT * dt;
    double P = -expm1(-x), K = L.sk / L.sig;
    double y = w * P * K;
    if (gout) {
        double Pp = exp(-x);
        /* energy axis: u = ln g (R, U) or ln(g - 1) (NR) */
        double du_dg = L.seg == SEG_NR ? 1.0 / gm1 : 1.0 / g;
        double dsig = L.dsig_du * du_dg, dsk = L.dsk_du * du_dg;
        double dbeta = 1.0 / (g * g * g * beta);
        double dx = ni * CLIGHT * dt * (dsig * beta + L.sig * dbeta);
        double dK = (dsk * L.sig - L.sk * dsig) / (L.sig * L.sig);
        double dyg = w * (Pp * dx * K + P * dK);
        double f = gY * dyg / g;
        gout[0] = f * px; gout[1] = f * py; gout[2] = f * pz;
        *gw = gY * P * K;
        for (int q = 0; q < 3; q++) {
            double ds, dk;
            if (L.seg == SEG_NR) {
                ds = L.dsig_a * G->dlnLd[q] + L.dsig_e * G->deta[q];
                dk = L.dsk_a * G->dlnLd[q] + L.dsk_e * G->deta[q];
            } else {
                ds = L.dsig_a * G->dlnLr[q];
                dk = L.dsk_a * G->dlnLr[q];
            }
            double dxq = x * G->dlnni[q] + ni * beta * CLIGHT * dt * ds;
            double dKq = (dk * L.sig - L.sk * ds) / (L.sig * L.sig);
            gcell[q] += gY * w * (Pp * dxq * K + P * dKq);
            if (gabs) {
                /* the size of the terms summed into gcell: the scale of its
                 * rounding error under any order of summation (tests only) */
                double ads, adk;
                if (L.seg == SEG_NR) {
                    ads = fabs(L.dsig_a * G->dlnLd[q]) + fabs(L.dsig_e * G->deta[q]);
                    adk = fabs(L.dsk_a * G->dlnLd[q]) + fabs(L.dsk_e * G->deta[q]);
                } else {
                    ads = fabs(L.dsig_a * G->dlnLr[q]);
                    adk = fabs(L.dsk_a * G->dlnLr[q]);
                }
                gabs[q] += fabs(gY * w) * (Pp * K * (fabs(x * G->dlnni[q]) + ni * beta * CLIGHT * dt * ads)
                                           + P * (adk * L.sig + L.sk * ads) / (L.sig * L.sig));
            }
        }
    }
    return y;
}

int or_expected_yield(const or_tables* t, int64_t n_cells, const double* Zs,
                      const double* n_e, const double* T_e, const int64_t* off,
                      const double* px, const double* py, const double* pz,
                      const double* w, double dt, double* Y, double* y_part, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_cells; c++) {
        double ni = n_e[c] / Zs[c];
        cellstate s; cell_init(t, Zs[c], ni, T_e[c], &s);
        double acc = 0.0;
        for (int64_t j = off[c]; j < off[c + 1]; j++) {
            double y = yield_one(t, &s, ni, px[j], py[j], pz[j], w[j], dt, NULL, NULL, NULL, NULL, NULL, 0.0);
            if (y_part) y_part[j] = y;
            acc += y;
        }
        Y[c] = acc;
    }
    return 0;
}

int or_expected_yield_backward(const or_tables* t, int64_t n_cells, const double* Zs,
                      const double* n_e, const double* T_e, const int64_t* off,
                      const double* px, const double* py, const double* pz,
                      const double* w, double dt, const double* gY,
                      double* gpx, double* gpy, double* gpz, double* gw,
                      double* gZs, double* gne, double* gTe, double* gabs, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_cells; c++) {
        double ni = n_e[c] / Zs[c];
        cellstate s; cell_init(t, Zs[c], ni, T_e[c], &s);
        cellgrad G; cell_jacobian(&s, n_e[c], &G);
        double gc[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
        for (int64_t j = off[c]; j < off[c + 1]; j++) {
            double g3[3], gwj;
            yield_one(t, &s, ni, px[j], py[j], pz[j], w[j], dt, g3, &gwj, gc, gabs ? ga : NULL, &G, gY[c]);
            gpx[j] = g3[0]; gpy[j] = g3[1]; gpz[j] = g3[2];
            if (gw) gw[j] = gwj;
        }
        gZs[c] = gc[0]; gne[c] = gc[1]; gTe[c] = gc[2];
        if (gabs) { gabs[3 * c] = ga[0]; gabs[3 * c + 1] = ga[1]; gabs[3 * c + 2] = ga[2]; }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* The step after.  Created particles are macro-particles of their     */
/* species (Sec. III.A): the photons a step creates convert in the     */
/* next one, and the electrons and positrons of a pair radiate and make */
/* pairs in turn (the chains of Sec. IV).  Merging appends a product    */
/* buffer to its population; rebinning gives a population new slabs.   */
/* Plain per-cell loops.                                                */
/* ------------------------------------------------------------------ */
static int32_t or_live(const or_species* s, int64_t c)
{
    int64_t cap = s->off[c + 1] - s->off[c];
    if (!s->count) return (int32_t)cap;
    int64_t n = s->count[c];
    if (n < 0) n = 0;
    return (int32_t)(n < cap ? n : cap);
}

void or_merge_species(int64_t n_cells, or_species* dst, or_species* src, int64_t* dropped)
{
    for (int64_t c = 0; c < n_cells; c++) {
        int32_t nd = or_live(dst, c), ns = or_live(src, c);
        int64_t cap = dst->off[c + 1] - dst->off[c];
        int64_t room = cap - nd;
        int32_t nk = (int32_t)(ns < room ? ns : room);
        for (int32_t i = 0; i < nk; i++) {
            int64_t a = src->off[c] + i, b = dst->off[c] + nd + i;
            dst->px[b] = src->px[a]; dst->py[b] = src->py[a]; dst->pz[b] = src->pz[a];
            dst->w[b] = src->w[a];
            if (dst->parent && src->parent) dst->parent[b] = src->parent[a];
        }
        dst->count[c] = nd + nk;
        src->count[c] = 0;
        if (dropped) dropped[c] = ns - nk;
    }
}

void or_rebin_offsets(int64_t n_cells, const or_species* s, int32_t headroom, int64_t* off_new)
{
    off_new[0] = 0;
    for (int64_t c = 0; c < n_cells; c++) off_new[c + 1] = off_new[c] + or_live(s, c) + headroom;
}

void or_rebin_copy(int64_t n_cells, const or_species* s, or_species* d)
{
    for (int64_t c = 0; c < n_cells; c++) {
        int32_t n = or_live(s, c);
        for (int32_t i = 0; i < n; i++) {
            int64_t a = s->off[c] + i, b = d->off[c] + i;
            d->px[b] = s->px[a]; d->py[b] = s->py[a]; d->pz[b] = s->pz[a]; d->w[b] = s->w[a];
            if (d->parent && s->parent) d->parent[b] = s->parent[a];
        }
        d->count[c] = n;
    }
}

