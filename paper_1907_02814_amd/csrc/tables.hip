// tables.hip -- construction of the cross-section tables on the device and
// the table part of the C ABI.
//
// One wavefront builds one table row: lane j integrates CDF panel j with
// Gauss-Legendre, then the panel integrals are accumulated in panel order
// into the cumulative distribution (numerical inversion of the cumulative
// distribution is how energies are sampled, Sec. III.A).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.hpp"

namespace cmc {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

TabView<double> view64(const cmc_tables_s* t) {
    TabView<double> v;
    for (int i = 0; i < grid::kNumArrays; ++i) v.a[i] = t->d64 + t->off[i];
    v.ax = t->ax; v.Z = t->Z; v.Ltf = t->Ltf; v.fc = t->fc;
    return v;
}

TabView<float> view32(const cmc_tables_s* t) {
    TabView<float> v;
    for (int i = 0; i < grid::kNumArrays; ++i) v.a[i] = t->d32 + t->off[i];
    v.ax = t->ax; v.Z = t->Z; v.Ltf = t->Ltf; v.fc = t->fc;
    return v;
}

namespace {

AxisDef make_axis(double u0, double u1, int n) {
    AxisDef a;
    a.u0 = u0; a.u1 = u1; a.n = n;
    a.du = (u1 - u0) / (n - 1);
    return a;
}

Axes make_axes() {
    Axes ax;
    ax.nr = make_axis(std::log(grid::kTminEv / grid::kMec2Ev), 0.0, grid::kNR);
    ax.rel = make_axis(std::log(2.0), std::log(100.0), grid::kRel);
    ax.ur = make_axis(std::log(100.0), std::log(grid::kTop), grid::kUR);
    ax.bh = make_axis(std::log(grid::kBHx0), std::log(grid::kTop - 2.0), grid::kBH);
    ax.tri = make_axis(std::log(3.0), std::log(grid::kTop), grid::kTri);
    ax.split = make_axis(std::log(4.0), std::log(grid::kTop), grid::kSplit);
    ax.L = make_axis(std::log(grid::kLmin), std::log(grid::kLmax), grid::kL);
    ax.eta = make_axis(0.0, 1.0, grid::kEta);
    return ax;
}

// Gauss-Legendre rule on [-1, 1]: roots of P_n by Newton's method, with the
// three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
void legendre_rule(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double r = std::cos(phys::kPi * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pkm1 = 1.0, pk = r;
            for (int k = 1; k < n; ++k) {
                const double pkp1 = ((2.0 * k + 1.0) * r * pk - k * pkm1) / (k + 1.0);
                pkm1 = pk; pk = pkp1;
            }
            dp = n * (r * pk - pkm1) / (r * r - 1.0);
            const double dr = pk / dp;
            r -= dr;
            if (std::fabs(dr) < 1e-16) break;
        }
        double pkm1 = 1.0, pk = r;
        for (int k = 1; k < n; ++k) {
            const double pkp1 = ((2.0 * k + 1.0) * r * pk - k * pkm1) / (k + 1.0);
            pkm1 = pk; pk = pkp1;
        }
        dp = n * (r * pk - pkm1) / (r * r - 1.0);
        x[n - 1 - i] = r;
        w[n - 1 - i] = 2.0 / ((1.0 - r * r) * dp * dp);
    }
}

constexpr long long kRowsRel = (long long)grid::kRel * grid::kL;
constexpr long long kRowsUR = (long long)grid::kUR * grid::kL;
constexpr long long kRowsNR = (long long)grid::kNR * grid::kEta * grid::kL;
constexpr long long kRowsBH = (long long)grid::kBH * grid::kL;
constexpr long long kRowsAll = kRowsRel + kRowsUR + kRowsNR + kRowsBH + grid::kTri + grid::kSplit;

struct BuildArgs {
    double* d;
    long long off[grid::kNumArrays];
    Axes ax;
    double Z, Ltf, fc;
    double gx[grid::kGauss], gw[grid::kGauss];
};

enum RowKind { kRowRel, kRowUR, kRowNR, kRowBH, kRowTri, kRowSplit };

struct RowDesc {
    int kind;
    long long r;          // row index within its array set
    double g1, g1m1, L, fc, etf, ed, Ld, Y, k, V, glo;
    bool degenerate;
};

__device__ inline double node(const AxisDef& a, int i) { return a.u0 + i * a.du; }

__device__ RowDesc describe(const BuildArgs& A, long long row) {
    RowDesc d;
    d.degenerate = false;
    d.fc = 0.0; d.etf = 1.0; d.ed = 0.0; d.Ld = 0.0; d.L = 0.0; d.k = 0.0; d.V = 0.0;
    d.glo = 0.0; d.Y = 0.0; d.g1 = 0.0; d.g1m1 = 0.0;
    if (row < kRowsRel + kRowsUR) {
        const bool ur = row >= kRowsRel;
        d.kind = ur ? kRowUR : kRowRel;
        d.r = ur ? row - kRowsRel : row;
        const int i = (int)(d.r / grid::kL), l = (int)(d.r % grid::kL);
        d.g1 = exp(node(ur ? A.ax.ur : A.ax.rel, i));
        d.g1m1 = d.g1 - 1.0;
        d.L = exp(node(A.ax.L, l));
        d.fc = ur ? A.fc : 0.0;
        d.Y = phys::brems_span(d.g1, d.g1m1);
        return d;
    }
    row -= kRowsRel + kRowsUR;
    if (row < kRowsNR) {
        d.kind = kRowNR; d.r = row;
        const int i = (int)(row / (grid::kEta * grid::kL));
        const int e = (int)((row / grid::kL) % grid::kEta), l = (int)(row % grid::kL);
        d.g1m1 = exp(node(A.ax.nr, i));
        d.g1 = 1.0 + d.g1m1;
        d.ed = (double)e / (grid::kEta - 1);
        d.etf = 1.0 - d.ed;
        d.Ld = exp(node(A.ax.L, l));
        d.Y = phys::brems_span(d.g1, d.g1m1);
        return d;
    }
    row -= kRowsNR;
    if (row < kRowsBH) {
        d.kind = kRowBH; d.r = row;
        const int i = (int)(row / grid::kL), l = (int)(row % grid::kL);
        d.k = 2.0 + exp(node(A.ax.bh, i));
        d.L = exp(node(A.ax.L, l));
        d.V = log(0.5 * d.k);
        return d;
    }
    row -= kRowsBH;
    if (row < grid::kTri) {
        d.kind = kRowTri; d.r = row;
        d.g1 = exp(node(A.ax.tri, (int)row));
        d.V = log(d.g1 - 1.0) - log(2.0);
        d.k = phys::trident_nr_bracket(d.g1);
        d.degenerate = !(d.V > 0.0);
        return d;
    }
    row -= grid::kTri;
    d.kind = kRowSplit; d.r = row;
    d.k = exp(node(A.ax.split, (int)row));          // pair energy
    d.glo = phys::split_low_edge(d.k);
    d.V = log(d.k / (2.0 * d.glo));
    d.degenerate = !(d.V > 0.0);
    return d;
}

__device__ double integrand(const BuildArgs& A, const RowDesc& d, double t, double& fk) {
    fk = 0.0;
    switch (d.kind) {
    case kRowRel:
    case kRowUR: {
        const phys::BremsPoint b = phys::brems_point(d.g1, d.g1m1, (1.0 - t) * d.Y);
        const double v = phys::brems_rel_dy(A.Z, d.g1, b, d.L, d.fc) * d.Y;
        fk = b.k * v;
        return v;
    }
    case kRowNR: {
        const phys::BremsPoint b = phys::brems_point(d.g1, d.g1m1, (1.0 - t) * (1.0 - t) * d.Y);
        const double v = phys::brems_nr_dy(A.Z, d.g1, d.g1m1, b, d.etf, d.ed, A.Ltf, d.Ld)
                       * 2.0 * (1.0 - t) * d.Y;
        fk = b.k * v;
        return v;
    }
    case kRowBH: {
        const double gp = exp(2.0 * t * d.V);
        return phys::bh_dsdgp(A.Z, d.k, gp, d.L) * gp * 2.0 * d.V;
    }
    case kRowTri: {
        const double gpair = exp(log(2.0) + t * d.V);
        return phys::trident_pair_shape(d.g1, d.k, gpair) * gpair * d.V;
    }
    default: {
        const double v = 2.0 * t * d.V;
        const double gplus = d.glo * exp(v), gminus = d.k - gplus;
        const double lg = log1p(d.glo * expm1(v) * (d.k - d.glo - gplus) / d.k);
        return (gplus * gplus + gminus * gminus + (2.0 / 3.0) * gplus * gminus) * lg * gplus * 2.0 * d.V;
    }
    }
}

__global__ __launch_bounds__(64) void k_build_rows(BuildArgs A) {
    const long long row = blockIdx.x;
    const int lane = threadIdx.x;
    const RowDesc d = describe(A, row);
    const bool half = d.kind == kRowBH || d.kind == kRowSplit;
    const int np = half ? grid::kPanels / 2 : grid::kPanels;
    __shared__ double part[grid::kPanels], partk[grid::kPanels], cum[grid::kRow];
    __shared__ double total_s, sk_s;
    double acc = 0.0, acck = 0.0;
    if (lane < np && !d.degenerate) {
        for (int g = 0; g < grid::kGauss; ++g) {
            const double t = (lane + 0.5 * (1.0 + A.gx[g])) / grid::kPanels;
            double fk;
            const double v = integrand(A, d, t, fk);
            acc += A.gw[g] * v;
            acck += A.gw[g] * fk;
        }
    }
    part[lane] = acc * (0.5 / grid::kPanels);
    partk[lane] = acck * (0.5 / grid::kPanels);
    __syncthreads();
    if (lane == 0) {
        double c = 0.0, ck = 0.0;
        cum[0] = 0.0;
        for (int j = 0; j < np; ++j) { c += part[j]; cum[j + 1] = c; ck += partk[j]; }
        total_s = half ? 2.0 * cum[grid::kPanels / 2] : cum[grid::kPanels];
        sk_s = ck;
    }
    __syncthreads();
    const double total = total_s;
    const bool flat = d.degenerate || !(total > 0.0);
    // CDF values j = lane and (lane 0) j = 64
    long long cdf_base, sig_idx = -1;
    int cdf_arr, sig_arr = -1, sk_arr = -1;
    switch (d.kind) {
    case kRowRel: cdf_arr = grid::kCdfR; sig_arr = grid::kSigR; sk_arr = grid::kSkR; break;
    case kRowUR: cdf_arr = grid::kCdfU; sig_arr = grid::kSigU; sk_arr = grid::kSkU; break;
    case kRowNR: cdf_arr = grid::kCdfN; sig_arr = grid::kSigN; sk_arr = grid::kSkN; break;
    case kRowBH: cdf_arr = grid::kCdfB; sig_arr = grid::kSigB; break;
    case kRowTri: cdf_arr = grid::kCdfT; break;
    default: cdf_arr = grid::kCdfS; break;
    }
    cdf_base = A.off[cdf_arr] + d.r * grid::kRow;
    if (sig_arr >= 0) sig_idx = d.r;
    for (int j = lane; j < grid::kRow; j += 64) {
        double v;
        if (flat) v = (double)j / grid::kPanels;
        else if (!half) v = cum[j] / total;
        else if (j <= grid::kPanels / 2) v = cum[j] / total;
        else v = 1.0 - cum[grid::kPanels - j] / total;
        A.d[cdf_base + j] = v;
    }
    if (lane == 0 && sig_idx >= 0) {
        A.d[A.off[sig_arr] + sig_idx] = flat ? 0.0 : total;
        if (sk_arr >= 0) A.d[A.off[sk_arr] + sig_idx] = flat ? 0.0 : sk_s;
    }
}

__global__ void k_to_fp32(const double* __restrict__ a, float* __restrict__ b, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        b[i] = (float)a[i];
}

}  // namespace
}  // namespace cmc

using namespace cmc;

extern "C" const char* cmc_last_error(void) { return cmc::g_err; }

extern "C" cmc_status cmc_build_tables(int32_t Z, void* stream, cmc_tables* out) {
    CMC_REQUIRE(out != nullptr, CMC_EINVAL, "cmc_build_tables: out is NULL");
    CMC_REQUIRE(Z >= 1 && Z <= 100, CMC_EINVAL, "cmc_build_tables: Z = %d outside [1, 100]", Z);
    *out = nullptr;
    cmc_tables_s* t = new cmc_tables_s();
    t->Z = Z;
    (void)hipGetDevice(&t->device);
    t->Ltf = 1.0 / (std::cbrt((double)Z) * phys::kAlpha);
    t->fc = phys::coulomb_correction((double)Z);
    t->ax = make_axes();
    long long o = 0;
    for (int i = 0; i < grid::kNumArrays; ++i) {
        t->off[i] = o;
        o += (grid::kCount[i] + 31) / 32 * 32;    // 256-byte aligned FP64 arrays
    }
    t->total = o;
    if (hipMalloc(&t->d64, sizeof(double) * o) != hipSuccess ||
        hipMalloc(&t->d32, sizeof(float) * o) != hipSuccess) {
        (void)hipGetLastError();
        if (t->d64) (void)hipFree(t->d64);
        delete t;
        set_error("cmc_build_tables: hipMalloc of %lld bytes failed", (long long)(12 * o));
        return CMC_ENOMEM;
    }
    hipStream_t s = as_stream(stream);
    (void)hipMemsetAsync(t->d64, 0, sizeof(double) * o, s);
    BuildArgs A;
    A.d = t->d64;
    for (int i = 0; i < grid::kNumArrays; ++i) A.off[i] = t->off[i];
    A.ax = t->ax; A.Z = Z; A.Ltf = t->Ltf; A.fc = t->fc;
    legendre_rule(grid::kGauss, A.gx, A.gw);
    hipLaunchKernelGGL(k_build_rows, dim3((unsigned)kRowsAll), dim3(64), 0, s, A);
    CMC_CHECK_LAUNCH("cmc_build_tables: k_build_rows");
    hipLaunchKernelGGL(k_to_fp32, dim3(1024), dim3(256), 0, s, t->d64, t->d32, o);
    CMC_CHECK_LAUNCH("cmc_build_tables: k_to_fp32");
    *out = t;
    return CMC_OK;
}

extern "C" cmc_status cmc_tables_free(cmc_tables t) {
    if (!t) return CMC_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(t->d64);
    (void)hipFree(t->d32);
    delete t;
    return CMC_OK;
}

extern "C" int64_t cmc_tables_size(cmc_tables t, int32_t which) {
    if (!t || which < 0 || which >= grid::kNumArrays) return -1;
    return grid::kCount[which];
}

extern "C" cmc_status cmc_tables_export(cmc_tables t, int32_t which, double* dst, int64_t n) {
    CMC_REQUIRE(t && dst, CMC_EINVAL, "cmc_tables_export: NULL argument");
    CMC_REQUIRE(which >= 0 && which < grid::kNumArrays, CMC_EINVAL, "cmc_tables_export: which = %d", which);
    CMC_REQUIRE(n == grid::kCount[which], CMC_EINVAL, "cmc_tables_export: n = %lld, expected %lld",
                (long long)n, grid::kCount[which]);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(dst, t->d64 + t->off[which], sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("cmc_tables_export: %s", hipGetErrorString(hipGetLastError()));
        return CMC_EDEVICE;
    }
    return CMC_OK;
}
