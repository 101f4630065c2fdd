// step.hip -- pairing and the Monte Carlo step (Sec. III.A) on the device.
//
// One workgroup of kThreads threads owns one cell at a time:
//   1. sums of weights (n_alpha = sum W, Sec. III.A) and the screening state;
//   2. for each pass (electron-ion, then photon-ion) both species are put in
//      Philox-key order in LDS (bucket by the top key bits, insertion sort
//      inside the buckets by (key, index)), n_ab = sum_j min(W_a, W_b);
//   3. pairs are processed in chunks of kThreads consecutive pair indices
//      that never hold the same mobile particle twice (a round of the
//      smaller species when that is the mobile one), so a particle reused by
//      later rounds is always handled by the same thread and sees its own
//      updates in pair order;
//   4. events append their products at slots given by a workgroup prefix
//      sum of ballots, i.e. in pair order, whatever the schedule;
//   5. photons converted by Bethe-Heitler are removed by a stable in-place
//      compaction; per-cell tallies are reduced in a fixed tree.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "philox.hpp"
#include "wave.hpp"

namespace cmc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// ------------------------------------------------------------------ helpers
// fixed-shape workgroup sum (deterministic for a given kThreads)
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
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

__device__ int block_or(int v, int* red) {
    const int w = threadIdx.x >> 6;
    const unsigned long long b = __ballot(v != 0);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = b != 0ull;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s |= red[i];
    __syncthreads();
    return s;
}

// exclusive prefix of a 0/1 flag over the workgroup in thread order;
// returns the prefix, writes the total
__device__ int block_flag_scan(bool f, int* red, int& total) {
    const unsigned long long b = __ballot(f);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int in_wave = __popcll(b & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) red[w] = __popcll(b);
    __syncthreads();
    int before = 0, t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) { if (i < w) before += red[i]; t += red[i]; }
    total = t;
    __syncthreads();
    return before + in_wave;
}

// inclusive prefix sum of a uint32 over the workgroup (thread order)
__device__ __forceinline__ uint32_t block_incl_scan_u32(uint32_t v, uint32_t* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) red[w] = v;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) if (i < w) before += red[i];
    __syncthreads();
    return v + before;
}

// exclusive scan of n uint32 counters in LDS (n <= 64 * kThreads), in place
__device__ void block_excl_scan_u32(uint32_t* a, int n, uint32_t* red) {
    const int per = (n + kThreads - 1) / kThreads;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += a[i];
    const uint32_t incl = block_incl_scan_u32(s, red);
    uint32_t run = incl - s;
    for (int i = lo; i < hi; ++i) { const uint32_t v = a[i]; a[i] = run; run += v; }
    __syncthreads();
}

__device__ __forceinline__ int bucket_bits(int n) {
    int b = 4;
    while (b < 12 && (1 << (b + 2)) < n) ++b;
    return b;
}

// perm[0..n) = indices 0..n-1 in increasing (Philox key, index) order
__device__ void key_order(int n, uint32_t cell, uint32_t tag, const Rng& rng, uint32_t* keys,
                          uint16_t* perm, uint32_t* bcnt, uint32_t* red) {
    if (n <= 0) return;
    const int bb = bucket_bits(n), nb = 1 << bb, sh = 32 - bb;
    for (int i = threadIdx.x; i < nb; i += kThreads) bcnt[i] = 0;
    __syncthreads();
    const int nq = (n + 3) >> 2;
    for (int q = threadIdx.x; q < nq; q += kThreads) {
        const U4 r = rng.draw((uint32_t)q, cell, tag);
        const uint32_t w4[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = 4 * q + u;
            if (i < n) { keys[i] = w4[u]; atomicAdd(&bcnt[w4[u] >> sh], 1u); }
        }
    }
    __syncthreads();
    block_excl_scan_u32(bcnt, nb, red);
    for (int i = threadIdx.x; i < n; i += kThreads) {
        const uint32_t pos = atomicAdd(&bcnt[keys[i] >> sh], 1u);
        perm[pos] = (uint16_t)i;
    }
    __syncthreads();
    // bcnt[b] now holds the end of bucket b
    for (int b = threadIdx.x; b < nb; b += kThreads) {
        const int lo = b ? (int)bcnt[b - 1] : 0, hi = (int)bcnt[b];
        for (int x = lo + 1; x < hi; ++x) {
            const uint16_t v = perm[x];
            const uint32_t kv = keys[v];
            int y = x - 1;
            while (y >= lo) {
                const uint16_t u = perm[y];
                const uint32_t ku = keys[u];
                if (ku < kv || (ku == kv && u < v)) break;
                perm[y + 1] = u;
                --y;
            }
            perm[y + 1] = v;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ shared layout
struct Smem {
    uint32_t* keys;
    uint16_t* pm;     // order of the mobile species (electrons / photons)
    uint16_t* pi;     // order of the ions
    uint32_t* bcnt;
    uint32_t* dead;   // bitmap of converted photons
};

__host__ __device__ inline int smem_buckets(int maxn) {
    int b = 4;
    while (b < 12 && (1 << (b + 2)) < maxn) ++b;
    return 1 << b;
}

__host__ __device__ inline size_t smem_bytes(int maxn) {
    const size_t n = (size_t)((maxn + 63) / 64 * 64);
    return n * 4 + n * 2 * 2 + (size_t)smem_buckets(maxn) * 4 + n / 8 + 64;
}

__device__ Smem carve(unsigned char* base, int maxn) {
    const size_t n = (size_t)((maxn + 63) / 64 * 64);
    Smem s;
    s.keys = reinterpret_cast<uint32_t*>(base);
    s.pm = reinterpret_cast<uint16_t*>(base + n * 4);
    s.pi = s.pm + n;
    s.bcnt = reinterpret_cast<uint32_t*>(base + n * 8);
    s.dead = s.bcnt + smem_buckets(maxn);
    return s;
}

// ------------------------------------------------------------------ step
struct SpeciesDev {
    const int64_t* off;
    int32_t* count;
    double *px, *py, *pz, *w;
    int64_t* parent;
};

struct StepArgs {
    SpeciesDev el, ph, io, ne, np;
    const double *Zs, *ni, *Te;
    const int64_t* cid;         // global cell indices (NULL: the position)
    int64_t n_cells;
    double dt, near_rel;
    Rng rng;
    uint32_t proc;
    int maxn;
    int64_t* ti;
    double* td;
    int32_t* status;
    const int32_t* list;        // non-NULL: process only the cells list[0 .. *list_n)
    const int32_t* list_n;
    const uint64_t* step_dev;   // non-NULL: the step number is read from device memory
};

// the cell word of the Philox counters of cell c: its global index
__device__ __forceinline__ uint32_t cell_word(const int64_t* cid, int64_t c) {
    return (uint32_t)(cid ? cid[c] : c);
}

// the generator of the step (step from device memory when it is there)
__device__ __forceinline__ Rng step_rng(const StepArgs& A) {
    Rng r = A.rng;
    if (A.step_dev) {
        const uint64_t s = *A.step_dev;
        r.step_lo = (uint32_t)s;
        r.step_hi = (uint32_t)(s >> 32);
    }
    return r;
}

// per-thread tallies (scalars: no dynamically indexed local arrays)
struct Tally {
    long long pairs_br, pairs_tr, pairs_bh, ev_br, ev_tr, ev_bh, near_br, near_tr, near_bh;
    long long drop_ph, drop_el, drop_po;
    double E_br, E_tr, E_bh, dE_el, dE_ph, W_br, W_tr, W_bh;
};

__device__ __forceinline__ int live(const SpeciesDev& s, int64_t c) {
    const int cap = (int)(s.off[c + 1] - s.off[c]);
    if (!s.count) return cap;
    const int n = s.count[c];
    return n < 0 ? 0 : (n > cap ? cap : n);
}

template <typename R>
struct CellShared {
    phys::Screen scr;
    CellTab<R> ct;          // lookup state of the per-pair path
    CellTab<double> ct64;   // lookup state of the (rare) event branch
};

template <typename R>
struct Elec { R g, gm1; double vrel; };

// electron: gamma, gamma - 1 in R and the speed |p| c / gamma in FP64
template <typename R>
__device__ __forceinline__ Elec<R> electron_p(double dx, double dy, double dz) {
    const R px = (R)dx, py = (R)dy, pz = (R)dz;
    const R p2 = px * px + py * py + pz * pz;
    Elec<R> e;
    e.g = Fast<R>::sqrt((R)1 + p2);
    e.gm1 = Fast<R>::div(p2, e.g + (R)1);
    const R pmag = Fast<R>::sqrt(p2);
    e.vrel = phys::kC * (double)Fast<R>::div(pmag, e.g);
    return e;
}

template <typename R>
__device__ __forceinline__ R photon_k(double px, double py, double pz) {
    const R qx = (R)px, qy = (R)py, qz = (R)pz;
    return Fast<R>::sqrt(qx * qx + qy * qy + qz * qz);
}

// ---- frame change of Sec. III.A: cross sections, sampling and products
// live in the rest frame of the ion of the pair, reached by the boost along
// the ion velocity.  u = gamma_i beta_i is the ion's proper velocity (the
// ions' px, py, pz); for ions at rest every transform is skipped.  All of it
// runs in FP64: the energy E' = gamma_i E - u.p cancels for particles that
// move with the ion.
struct Ion { double ux, uy, uz, gi; bool mov; };

__device__ __forceinline__ Ion ion_at(const SpeciesDev& io, int64_t ii) {
    Ion b{0.0, 0.0, 0.0, 1.0, false};
    if (io.px) {
        b.ux = io.px[ii]; b.uy = io.py[ii]; b.uz = io.pz[ii];
        b.gi = sqrt(1.0 + b.ux * b.ux + b.uy * b.uy + b.uz * b.uz);
        b.mov = true;
    }
    return b;
}

// (E, p) -> (E', p') in the ion frame: E' = gamma_i E - u.p,
// p' = p + (u.p / (gamma_i + 1) - E) u
__device__ __forceinline__ double to_ion(const Ion& b, double E, double px, double py, double pz,
                                         double& qx, double& qy, double& qz) {
    const double up = b.ux * px + b.uy * py + b.uz * pz;
    const double s = up / (b.gi + 1.0) - E;
    qx = px + s * b.ux; qy = py + s * b.uy; qz = pz + s * b.uz;
    return b.gi * E - up;
}

// the inverse, momentum only: p = p' + (u.p' / (gamma_i + 1) + E') u
__device__ __forceinline__ void from_ion(const Ion& b, double E, double qx, double qy, double qz,
                                         double& px, double& py, double& pz) {
    const double up = b.ux * qx + b.uy * qy + b.uz * qz;
    const double s = up / (b.gi + 1.0) + E;
    px = qx + s * b.ux; py = qy + s * b.uy; pz = qz + s * b.uz;
}

// a mobile particle seen from the ion, FP64: the energy gamma' (electron) or
// k' (photon), gamma' - 1, |p'| and p'; E is the lab energy
struct Frame { double g, gm1, pm, qx, qy, qz, E; };

__device__ __forceinline__ Frame electron_frame(const Ion& b, double px, double py, double pz) {
    Frame f;
    const double p2 = px * px + py * py + pz * pz;
    f.E = sqrt(1.0 + p2);
    if (!b.mov) {
        f.g = f.E; f.gm1 = p2 / (f.E + 1.0); f.pm = sqrt(p2);
        f.qx = px; f.qy = py; f.qz = pz;
        return f;
    }
    f.g = to_ion(b, f.E, px, py, pz, f.qx, f.qy, f.qz);
    const double q2 = f.qx * f.qx + f.qy * f.qy + f.qz * f.qz;
    f.gm1 = q2 / (sqrt(1.0 + q2) + 1.0);
    f.pm = sqrt(q2);
    return f;
}

__device__ __forceinline__ Frame photon_frame(const Ion& b, double px, double py, double pz) {
    Frame f;
    f.E = sqrt(px * px + py * py + pz * pz);
    f.gm1 = 0.0;
    if (!b.mov) {
        f.g = f.pm = f.E; f.qx = px; f.qy = py; f.qz = pz;
        return f;
    }
    f.g = f.pm = to_ion(b, f.E, px, py, pz, f.qx, f.qy, f.qz);
    return f;
}

// eq:proba2: the ion-frame electron for the per-pair test, with the rate
// factor gamma' v' / (gamma_e gamma_i) = c |p'| / (gamma_e gamma_i)
template <typename R>
__device__ __forceinline__ Elec<R> electron_moving(const Frame& f, const Ion& b) {
    Elec<R> e;
    e.g = (R)f.g;
    e.gm1 = (R)f.gm1;
    e.vrel = phys::kC * f.pm / (f.E * b.gi);
    return e;
}

// the photon's flux factor k' c / (k gamma_i) (c for ions at rest)
__device__ __forceinline__ double photon_flux(const Frame& f, const Ion& b) {
    return b.mov ? phys::kC * f.pm / (f.E * b.gi) : phys::kC;
}

// lab momentum of a product with ion-frame energy E and momentum magnitude
// mag along the parent's ion-frame direction
__device__ __forceinline__ void lab_along(const Ion& b, const Frame& f, double E, double mag,
                                          double& x, double& y, double& z) {
    if (!b.mov) {
        const double s = mag / f.pm;
        x = f.qx * s; y = f.qy * s; z = f.qz * s;
        return;
    }
    const double r = 1.0 / f.pm;
    from_ion(b, E, (f.qx * r) * mag, (f.qy * r) * mag, (f.qz * r) * mag, x, y, z);
}

// lab energy change of an electron that loses dE in the ion frame (its
// momentum there goes from pm to pf along the same direction):
// gamma_i dE + u.n (pf - pm), with pf - pm = dE (gf + g) / (pf + pm) so that
// nothing cancels when dE << gamma
__device__ __forceinline__ double lab_energy_change(const Ion& b, const Frame& f, double dE, double gf, double pf) {
    if (!b.mov) return dE;
    const double r = 1.0 / f.pm;
    const double un = b.ux * (f.qx * r) + b.uy * (f.qy * r) + b.uz * (f.qz * r);
    return b.gi * dE + un * (dE * (gf + f.g) / (pf + f.pm));
}

// all tallies of the cell reduced in one pass: wavefront sums, then the
// waves' partials summed in wave order by one thread (fixed shape)
__device__ void write_tallies(const StepArgs& A, int64_t c, const Tally& t, double nab_ei,
                              double nab_gi, long long* redl, double* redd) {
    long long iv[CMC_NI] = {t.pairs_br, t.pairs_tr, t.pairs_bh, t.ev_br, t.ev_tr, t.ev_bh,
                            t.near_br, t.near_tr, t.near_bh, t.drop_ph, t.drop_el, t.drop_po};
    double dv[8] = {t.E_br, t.E_tr, t.E_bh, t.dE_el, t.dE_ph, t.W_br, t.W_tr, t.W_bh};
    // (a thread's counts are at most its share of one cell's pairs)
#pragma unroll
    for (int q = 0; q < CMC_NI; ++q) iv[q] = wave_sum_i32((int)iv[q]);
#pragma unroll
    for (int q = 0; q < 8; ++q) dv[q] = wave_sum(dv[q]);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int q = 0; q < CMC_NI; ++q) redl[w * CMC_NI + q] = iv[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) redd[w * 8 + q] = dv[q];
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < CMC_NI) {
        long long s = 0;
        for (int i = 0; i < kWaves; ++i) s += redl[i * CMC_NI + q];
        A.ti[c * CMC_NI + q] = s;
    } else if (q < CMC_NI + 8) {
        const int r = q - CMC_NI;
        double s = redd[r];
        for (int i = 1; i < kWaves; ++i) s += redd[i * 8 + r];
        A.td[c * CMC_ND + CMC_D_E_BR + r] = s;
    } else if (q == CMC_NI + 8) {
        A.td[c * CMC_ND + CMC_D_NAB_EI] = nab_ei;
        A.td[c * CMC_ND + CMC_D_NAB_GI] = nab_gi;
    }
    __syncthreads();
}

template <typename R>
struct CollideShared {   // static LDS of the sequential per-cell step
    double redd[kWaves * 8];
    long long redl[kWaves * CMC_NI];
    int redi[kWaves];
    uint32_t redu[kWaves];
    CellShared<R> cs;
};

// The whole step of one cell, pairs in order (the sequential semantics of
// the method), by a workgroup of kThreads.  R is the arithmetic of the
// per-pair path (table interpolation of the cross sections, gamma, beta);
// events sample their energies from the FP64 tables T64 in FP64 in both
// forms.
template <typename R>
__device__ __forceinline__ void collide_cell(const StepArgs& A, const TabView<R>& T, const TabView<double>& T64, const Rng& rng,
                             int64_t c, const Smem& S, CollideShared<R>& sh) {
    double* redd = sh.redd;
    long long* redl = sh.redl;
    int* redi = sh.redi;
    uint32_t* redu = sh.redu;
    CellShared<R>& cs = sh.cs;
    const int tid = threadIdx.x;
    const uint32_t cell = cell_word(A.cid, c);
    const int Ne = live(A.el, c), Ng0 = live(A.ph, c), Ni = live(A.io, c);
    const int64_t e0 = A.el.off[c], g0 = A.ph.off[c], i0 = A.io.off[c];
    const double Zs = A.Zs[c], nic = A.ni[c], Te = A.Te[c];
    Tally t = {};
    bool skip = false;
    int st = 0;
    if (!(Zs >= 0.0 && Zs <= T.Z && nic > 0.0 && Te >= 0.0 && isfinite(nic) && isfinite(Te))) {
        st = CMC_ST_BAD_CELL; skip = true;
    } else if (Ne > A.maxn || Ng0 > A.maxn || Ni > A.maxn) {
        st = CMC_ST_TOO_LARGE; skip = true;
    }
    // densities and weight check
    double se = 0.0, sg = 0.0, si = 0.0;
    int bad = 0;
    if (!skip) {
        for (int a = tid; a < Ne; a += kThreads) { const double w = A.el.w[e0 + a]; se += w; bad |= !(w >= 0.0) || !isfinite(w); }
        for (int a = tid; a < Ng0; a += kThreads) { const double w = A.ph.w[g0 + a]; sg += w; bad |= !(w >= 0.0) || !isfinite(w); }
        for (int a = tid; a < Ni; a += kThreads) { const double w = A.io.w[i0 + a]; si += w; bad |= !(w >= 0.0) || !isfinite(w); }
        if (tid == 0) {
            cs.scr = phys::screening(T.Z, Zs, nic, Te);
            cs.ct = cell_tab<R>(cs.scr, T.ax);
            cs.ct64 = cell_tab<double>(cs.scr, T.ax);
        }
    }
    const double n_e = block_sum(se, redd), n_g = block_sum(sg, redd), n_I = block_sum(si, redd);
    if (!skip && block_or(bad, redi)) { st = CMC_ST_BAD_WEIGHT; skip = true; }
    double nab_ei = 0.0, nab_gi = 0.0;
    if (skip) {
        if (tid == 0) atomicOr(A.status, st);
        write_tallies(A, c, t, 0.0, 0.0, redl, redd);
        return;
    }
    const CellTab<R> ct = cs.ct;
    const CellTab<double> ct64 = cs.ct64;
    bool high_any = false;

    // ---------------------------------------------- electron-ion pass
    int ph_count = Ng0;   // photons in the species after Bremsstrahlung appends
    const int cap_ph = (int)(A.ph.off[c + 1] - g0);
    int cnt_ne = A.ne.count[c], cnt_np = A.np.count[c];
    const int cap_ne = (int)(A.ne.off[c + 1] - A.ne.off[c]), cap_np = (int)(A.np.off[c + 1] - A.np.off[c]);
    if ((A.proc & (CMC_BREMS | CMC_TRIDENT)) && Ne > 0 && Ni > 0) {
        key_order(Ne, cell, kTagKeyE, rng, S.keys, S.pm, S.bcnt, redu);
        key_order(Ni, cell, kTagKeyIE, rng, S.keys, S.pi, S.bcnt, redu);
        const int N = Ne > Ni ? Ne : Ni;
        double part = 0.0;
        for (int j = tid; j < N; j += kThreads) {
            const double we = A.el.w[e0 + S.pm[j % Ne]], wi = A.io.w[i0 + S.pi[j % Ni]];
            part += we < wi ? we : wi;
        }
        nab_ei = block_sum(part, redd);
        const double coef = n_e * n_I / nab_ei;
        const int run = Ne >= Ni ? N : Ne;          // pairs in a run never repeat an electron
        for (int r0 = (nab_ei > 0.0 ? 0 : N); r0 < N; r0 += run) {
            const int rend = min(N, r0 + run);
            for (int base = r0; base < rend; base += kThreads) {
                const int j = base + tid;
                const bool act = j < rend;
                bool f_ph = false, f_tr = false;
                double kx = 0, ky = 0, kz = 0, pxm = 0, pym = 0, pzm = 0, pxp = 0, pyp = 0, pzp = 0, We = 0;
                int64_t ie = 0;
                if (act) {
                    const int me = S.pm[j % Ne];
                    ie = e0 + me;
                    const int64_t ii = i0 + S.pi[j % Ni];
                    // the pair's draws: keyed by its electron and its repetition
                    const uint32_t dk = (uint32_t)(me + (j / Ne) * Ne);
                    We = A.el.w[ie];
                    const double Wi = A.io.w[ii];
                    const double Pej = Wi / (We > Wi ? We : Wi);
                    double px = A.el.px[ie], py = A.el.py[ie], pz = A.el.pz[ie];
                    const Ion b = ion_at(A.io, ii);
                    bool moved = false;
                    for (int proc = 0; proc < 2; ++proc) {
                        const uint32_t bit = proc == 0 ? CMC_BREMS : CMC_TRIDENT;
                        if (!(A.proc & bit)) continue;
                        if (proc == 0) t.pairs_br++; else t.pairs_tr++;
                        // the electron (after this pair's Bremsstrahlung for Trident) seen from the ion
                        const Frame f = electron_frame(b, px, py, pz);
                        const Elec<R> e = b.mov ? electron_moving<R>(f, b) : electron_p<R>(px, py, pz);
                        const R g = e.g, gm1 = e.gm1;
                        R sig;
                        BremsLook<R> BL;
                        bool high = false;
                        if (proc == 0) { BL = brems_lookup<R>(T, ct, g, gm1, high); sig = BL.sig; }
                        else sig = (R)phys::trident_sigma(T.Z, (double)g);
                        high_any |= high;
                        if (!(sig > (R)0)) continue;
                        // eq:proba3 with gamma' v' = c |p'| (eq:proba2)
                        const double x = coef * (double)sig * e.vrel * A.dt;
                        const double P = -expm1(-x);
                        double U1, U2;
                        accept_uniforms(rng, dk, cell, proc == 0 ? kTagAccBr : kTagAccTr, proc == 0 ? kTagHiBr : kTagHiTr,
                                        U1, U2);
                        if (fabs(U1 - P) <= A.near_rel * P) { if (proc == 0) t.near_br++; else t.near_tr++; }
                        if (!(U1 < P && U2 < Pej)) continue;
                        const U4 q = rng.draw(dk, cell, proc == 0 ? kTagSmpBr : kTagSmpTr);
                        const double xi1 = u53(q.x, q.y), xi2 = u53(q.z, q.w);
                        if (proc == 0) t.ev_br++; else t.ev_tr++;
                        moved = true;
                        // event kinematics in FP64, in the ion frame
                        if (proc == 0) {
                            bool hi2;
                            const BremsLook<double> BLd = brems_lookup<double, false>(T64, ct64, f.g, f.gm1, hi2);
                            double k, g2, g2m1;
                            brems_sample<double>(T64, ct64, BLd, f.g, f.gm1, xi1, k, g2, g2m1);
                            // photon along the electron, which keeps its direction
                            const double pf = sqrt(g2m1 * (g2 + 1.0));
                            lab_along(b, f, k, k, kx, ky, kz);
                            lab_along(b, f, g2, pf, px, py, pz);
                            t.E_br += We * sqrt(kx * kx + ky * ky + kz * kz);
                            // energy change from -k (exact in the ion frame): the
                            // difference of two Lorentz factors would cancel for k << gamma
                            t.dE_el += We * lab_energy_change(b, f, -k, g2, pf);
                            t.W_br += We;
                            f_ph = true;
                        } else {
                            double gpair, gpl, gmi, gfm1;
                            trident_sample<double>(T64, f.g, f.gm1, xi1, xi2, gpair, gpl, gmi, gfm1);
                            const double gf = gfm1 + 1.0;
                            const double pf = sqrt(gfm1 * (gf + 1.0));
                            const double pplus = sqrt((gpl - 1.0) * (gpl + 1.0));
                            const double pminus = sqrt((gmi - 1.0) * (gmi + 1.0));
                            lab_along(b, f, gpl, pplus, pxp, pyp, pzp);
                            lab_along(b, f, gmi, pminus, pxm, pym, pzm);
                            lab_along(b, f, gf, pf, px, py, pz);
                            const double gpl_l = sqrt(1.0 + pxp * pxp + pyp * pyp + pzp * pzp);
                            const double gmi_l = sqrt(1.0 + pxm * pxm + pym * pym + pzm * pzm);
                            t.E_tr += We * (gpl_l + gmi_l);
                            t.dE_el += We * lab_energy_change(b, f, -gpair, gf, pf);
                            t.W_tr += We;
                            f_tr = true;
                        }
                    }
                    if (moved) { A.el.px[ie] = px; A.el.py[ie] = py; A.el.pz[ie] = pz; }
                }
                // ordered appends (pair order within the chunk)
                int tot_ph, tot_tr;
                const int o_ph = block_flag_scan(f_ph, redi, tot_ph);
                const int o_tr = block_flag_scan(f_tr, redi, tot_tr);
                if (f_ph) {
                    const int slot = ph_count + o_ph;
                    if (slot < cap_ph) {
                        const int64_t at = g0 + slot;
                        A.ph.px[at] = kx; A.ph.py[at] = ky; A.ph.pz[at] = kz; A.ph.w[at] = We;
                        if (A.ph.parent) A.ph.parent[at] = ie;
                    } else { t.drop_ph++; }
                }
                if (f_tr) {
                    const int s1 = cnt_ne + o_tr, s2 = cnt_np + o_tr;
                    if (s1 < cap_ne) {
                        const int64_t at = A.ne.off[c] + s1;
                        A.ne.px[at] = pxm; A.ne.py[at] = pym; A.ne.pz[at] = pzm; A.ne.w[at] = We;
                        if (A.ne.parent) A.ne.parent[at] = ie;
                    } else { t.drop_el++; }
                    if (s2 < cap_np) {
                        const int64_t at = A.np.off[c] + s2;
                        A.np.px[at] = pxp; A.np.py[at] = pyp; A.np.pz[at] = pzp; A.np.w[at] = We;
                        if (A.np.parent) A.np.parent[at] = ie;
                    } else { t.drop_po++; }
                }
                ph_count = min(cap_ph, ph_count + tot_ph);
                cnt_ne = min(cap_ne, cnt_ne + tot_tr);
                cnt_np = min(cap_np, cnt_np + tot_tr);
            }
        }
    }

    // ---------------------------------------------- photon-ion pass
    bool any_dead = false;
    if ((A.proc & CMC_BH) && Ng0 > 0 && Ni > 0) {
        for (int i = tid; i < (Ng0 + 31) / 32; i += kThreads) S.dead[i] = 0u;
        key_order(Ng0, cell, kTagKeyG, rng, S.keys, S.pm, S.bcnt, redu);
        key_order(Ni, cell, kTagKeyIG, rng, S.keys, S.pi, S.bcnt, redu);
        const int N = Ng0 > Ni ? Ng0 : Ni;
        double part = 0.0;
        for (int j = tid; j < N; j += kThreads) {
            const double wg = A.ph.w[g0 + S.pm[j % Ng0]], wi = A.io.w[i0 + S.pi[j % Ni]];
            part += wg < wi ? wg : wi;
        }
        nab_gi = block_sum(part, redd);
        const double coef = n_g * n_I / nab_gi;
        const int run = Ng0 >= Ni ? N : Ng0;
        int killed = 0;
        for (int r0 = (nab_gi > 0.0 ? 0 : N); r0 < N; r0 += run) {
            const int rend = min(N, r0 + run);
            for (int base = r0; base < rend; base += kThreads) {
                const int j = base + tid;
                bool f_bh = false;
                double pxm = 0, pym = 0, pzm = 0, pxp = 0, pyp = 0, pzp = 0, Wg = 0;
                int64_t ig = 0;
                if (j < rend) {
                    const int lg = S.pm[j % Ng0];
                    const bool dead = (S.dead[lg >> 5] >> (lg & 31)) & 1u;
                    if (!dead) {
                        ig = g0 + lg;
                        const int64_t ii = i0 + S.pi[j % Ni];
                        const uint32_t dk = (uint32_t)(lg + (j / Ng0) * Ng0);   // keyed by the photon and its repetition
                        t.pairs_bh++;
                        Wg = A.ph.w[ig];
                        const double Wi = A.io.w[ii];
                        const double Pej = Wi / (Wg > Wi ? Wg : Wi);
                        const double qx = A.ph.px[ig], qy = A.ph.py[ig], qz = A.ph.pz[ig];
                        const Ion b = ion_at(A.io, ii);
                        const Frame f = photon_frame(b, qx, qy, qz);
                        const R k = b.mov ? (R)f.g : photon_k<R>(qx, qy, qz);
                        int ik; R wk; bool high;
                        const R sig = bh_lookup<R>(T, ct, k, ik, wk, high);
                        high_any |= high;
                        if (sig > (R)0) {
                            // eq:proba3 for photons: gamma -> k', v' -> c, flux k' c/(k gamma_i)
                            const double x = coef * (double)sig * photon_flux(f, b) * A.dt;
                            const double P = -expm1(-x);
                            double U1, U2;
                            accept_uniforms(rng, dk, cell, kTagAccBh, kTagHiBh, U1, U2);
                            if (fabs(U1 - P) <= A.near_rel * P) t.near_bh++;
                            if (U1 < P && U2 < Pej) {
                                const U4 q = rng.draw(dk, cell, kTagSmpBh);
                                double gpl, gmi;
                                int ikd; double wkd; bool hi2;
                                bh_lookup<double>(T64, ct64, f.g, ikd, wkd, hi2);
                                bh_sample<double>(T64, ct64, f.g, ikd, wkd, u53(q.x, q.y), gpl, gmi);
                                // the pair travels along the photon (ion frame)
                                const double pplus = sqrt((gpl - 1.0) * (gpl + 1.0));
                                const double pminus = sqrt((gmi - 1.0) * (gmi + 1.0));
                                lab_along(b, f, gpl, pplus, pxp, pyp, pzp);
                                lab_along(b, f, gmi, pminus, pxm, pym, pzm);
                                const double gpl_l = sqrt(1.0 + pxp * pxp + pyp * pyp + pzp * pzp);
                                const double gmi_l = sqrt(1.0 + pxm * pxm + pym * pym + pzm * pzm);
                                atomicOr(&S.dead[lg >> 5], 1u << (lg & 31));
                                t.ev_bh++;
                                t.E_bh += Wg * (gpl_l + gmi_l);
                                t.dE_ph += -Wg * f.E;
                                t.W_bh += Wg;
                                f_bh = true;
                            }
                        }
                    }
                }
                int tot;
                const int o = block_flag_scan(f_bh, redi, tot);
                if (f_bh) {
                    const int s1 = cnt_ne + o, s2 = cnt_np + o;
                    if (s1 < cap_ne) {
                        const int64_t at = A.ne.off[c] + s1;
                        A.ne.px[at] = pxm; A.ne.py[at] = pym; A.ne.pz[at] = pzm; A.ne.w[at] = Wg;
                        if (A.ne.parent) A.ne.parent[at] = ig;
                    } else { t.drop_el++; }
                    if (s2 < cap_np) {
                        const int64_t at = A.np.off[c] + s2;
                        A.np.px[at] = pxp; A.np.py[at] = pyp; A.np.pz[at] = pzp; A.np.w[at] = Wg;
                        if (A.np.parent) A.np.parent[at] = ig;
                    } else { t.drop_po++; }
                }
                killed += tot;
                cnt_ne = min(cap_ne, cnt_ne + tot);
                cnt_np = min(cap_np, cnt_np + tot);
            }
        }
        any_dead = killed > 0;
    }

    // ---------------------------------------------- photon compaction
    if (any_dead) {
        int wpos = 0;
        for (int base = 0; base < ph_count; base += kThreads) {
            const int a = base + tid;
            bool keep = false;
            double vx = 0, vy = 0, vz = 0, vw = 0;
            int64_t par = -1;
            if (a < ph_count) {
                keep = !(a < Ng0 && ((S.dead[a >> 5] >> (a & 31)) & 1u));
                if (keep) {
                    vx = A.ph.px[g0 + a]; vy = A.ph.py[g0 + a]; vz = A.ph.pz[g0 + a]; vw = A.ph.w[g0 + a];
                    if (A.ph.parent) par = A.ph.parent[g0 + a];
                }
            }
            int tot;
            const int o = block_flag_scan(keep, redi, tot);   // barrier: all reads precede writes
            if (keep) {
                const int64_t at = g0 + wpos + o;
                A.ph.px[at] = vx; A.ph.py[at] = vy; A.ph.pz[at] = vz; A.ph.w[at] = vw;
                if (A.ph.parent) A.ph.parent[at] = par;
            }
            wpos += tot;
            __syncthreads();
        }
        ph_count = wpos;
    }

    // ---------------------------------------------- counts, tallies
    if (high_any) atomicOr(A.status, CMC_ST_GAMMA_HIGH);
    if (t.drop_ph + t.drop_el + t.drop_po) atomicOr(A.status, CMC_ST_OVERFLOW);
    if (tid == 0) {
        if (A.ph.count) A.ph.count[c] = ph_count;
        A.ne.count[c] = cnt_ne;
        A.np.count[c] = cnt_np;
    }
    write_tallies(A, c, t, nab_ei, nab_gi, redl, redd);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_collide(StepArgs A, TabView<R> T, TabView<double> T64) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ CollideShared<R> sh;
    const Smem S = carve(smem_raw, A.maxn);
    const Rng rng = step_rng(A);
    const int64_t n_items = A.list ? (int64_t)*A.list_n : A.n_cells;
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t c = A.list ? (int64_t)A.list[item] : item;
        collide_cell<R>(A, T, T64, rng, c, S, sh);
    }
}


// ------------------------------------------------------------------ fast path
// The step is split in launches.  k_cell_state computes the screening
// state of every cell and clears its tallies.  k_pass (one launch per pass)
// tests every pair of a cell with the particles as they are at the start of
// the step; this is exact whenever no particle used by a later pair of the
// same pass changes before that pair, i.e. when every event falls on the
// last pair of its particle.  Tests the bound on P cannot settle are listed
// per cell; k_events settles them and applies the events of the cell in
// pair order.  Cells where the start-of-step reading does not hold (an event
// on a particle used again, more open pairs than kCandCap, more particles
// than the pass kernel's LDS) are redone by k_events with the sequential
// per-cell step above (collide_cell).
constexpr int kCandCap = 64;     // open pairs per cell (both passes)
constexpr int kStagePh = 1024;   // photons the event kernel stages in LDS per cell
// per-cell flags of a step: kFlagWeightsOk, set by the electron-ion pass,
// says every weight of the cell is valid and its ion sum is in ionsum
// (kFlagIonsSame: the ions share one weight), so that the photon-ion pass
// reads neither the ions' nor the electrons' weights again; kFlagDone0,
// kFlagDone1: the stream kernel has run the cell's electron-ion pass, its
// photon-ion pass
enum : int32_t { kFlagSlow = 1, kFlagListed = 2, kFlagBig0 = 4, kFlagBig1 = 8, kFlagWeightsOk = 16, kFlagIonsSame = 32,
                 kFlagDone0 = 64, kFlagDone1 = 128 };
enum : uint32_t { kEvBr = 1, kEvTrPending = 2, kEvTr = 4, kEvBh = 8 };

struct CellState {
    CellTab<double> d;
    CellTab<float> f;
    int32_t status;                  // CMC_ST_BAD_CELL or 0
};

// list counters of a step (Work::counters), cleared by k_cell_state
enum : int {
    kCntEv = 0,      // cells listed for the event kernels (list_ev)
    kCntBig0 = 1,    // electron-ion passes deferred to the large-LDS launch (list_big[0])
    kCntBig1 = 2,    // photon-ion passes deferred (list_big[1])
    kCntWg = 3,      // listed cells the wavefront event kernel hands to the workgroup one (list_wg)
    kCntRest = 4,    // cells the stream kernel leaves to the pass kernel (marked in list_rest)
    kCntLane = 5,    // cells the stream kernel lists for the lane event kernel (list_lane)
    kNumCnt = 8
};

struct Work {
    CellState* cs;
    int32_t* flags;                  // kFlagSlow: the sequential kernel runs the cell
    int32_t* ncand;                  // open pairs pushed per cell
    double* coef;                    // n_a n_b / n_ab per cell and pass
    double* ionsum;                  // canonical sum of the ion weights (with kFlagWeightsOk)
    uint64_t* step;                  // step number of the current step
    int32_t* counters;               // kNumCnt list lengths
    int32_t* list_ev;                // cells with open pairs or flagged for the sequential step
    int32_t* list_wg;                // listed cells that need the workgroup event kernel
    int32_t* list_big[2];            // per pass: cells whose pass needs more LDS than the first launch has
    int32_t* queue;                  // the cells in decreasing order of cost (batched schedule)
    int32_t* list_rest;              // per item of the stream kernel's walk: its cell if a pass is left, else -1
    int32_t* list_lane;              // listed cells for the lane event kernel (k_events_lane)
    uint64_t* cand;                  // [n_cells][kCandCap] open pairs
};

__host__ __device__ constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

__host__ __device__ constexpr size_t work_bytes(int64_t n) {
    return align256(sizeof(CellState) * n) + align256(4 * n) + align256(4 * n) +
           align256(16 * n) + align256(8 * n) + align256(8) + align256(4 * kNumCnt) + 7 * align256(4 * n) +
           align256(8 * (size_t)n * kCandCap);
}

inline Work carve_work(void* base, int64_t n) {
    unsigned char* p = static_cast<unsigned char*>(base);
    Work w;
    w.cs = reinterpret_cast<CellState*>(p); p += align256(sizeof(CellState) * n);
    w.flags = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.ncand = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.coef = reinterpret_cast<double*>(p); p += align256(16 * n);
    w.ionsum = reinterpret_cast<double*>(p); p += align256(8 * n);
    w.step = reinterpret_cast<uint64_t*>(p); p += align256(8);
    w.counters = reinterpret_cast<int32_t*>(p); p += align256(4 * kNumCnt);
    w.list_ev = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.list_wg = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.list_big[0] = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.list_big[1] = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.queue = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.list_rest = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.list_lane = reinterpret_cast<int32_t*>(p); p += align256(4 * n);
    w.cand = reinterpret_cast<uint64_t*>(p);
    return w;
}

__device__ __forceinline__ uint64_t ev_pack(int pass, int j, int mi, int ii, uint32_t kind) {
    return (uint64_t)(uint32_t)j | ((uint64_t)(uint32_t)mi << 16) | ((uint64_t)(uint32_t)ii << 32) |
           ((uint64_t)(kind | (uint32_t)pass << 7) << 48);
}
__device__ __forceinline__ int ev_j(uint64_t r) { return (int)(r & 0xFFFF); }
__device__ __forceinline__ int ev_m(uint64_t r) { return (int)((r >> 16) & 0xFFFF); }
__device__ __forceinline__ int ev_i(uint64_t r) { return (int)((r >> 32) & 0xFFFF); }
__device__ __forceinline__ uint32_t ev_kind(uint64_t r) { return (uint32_t)(r >> 48) & 0x7F; }
__device__ __forceinline__ int ev_pass(uint64_t r) { return (int)((r >> 55) & 1); }
__device__ __forceinline__ uint32_t ev_key(uint64_t r) { return ((uint32_t)ev_pass(r) << 16) | (uint32_t)ev_j(r); }

// screening state of every cell; clears the cell's tallies and work
// counters and the list counters of the step
// The step number: from the device counter when there is one (which then
// advances, so that a captured graph runs the next step on every replay),
// else from the host.
__global__ void k_cell_state(const double* Zs, const double* ni, const double* Te, int64_t n, double Z,
                             Axes ax, Work W, int64_t* ti, double* td, int32_t* status, uint64_t* counter,
                             uint64_t host_step, int advance) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t st = counter ? *counter : host_step;
        W.step[0] = st;
        if (counter && advance) *counter = st + 1;
    }
    if (blockIdx.x == 0 && threadIdx.x < kNumCnt) W.counters[threadIdx.x] = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const double z = Zs[c], d = ni[c], t = Te[c];
        CellState s = {};
        W.flags[c] = 0;
        W.ncand[c] = 0;
        for (int q = 0; q < CMC_NI; ++q) ti[c * CMC_NI + q] = 0;
        for (int q = 0; q < CMC_ND; ++q) td[c * CMC_ND + q] = 0.0;
        if (!(z >= 0.0 && z <= Z && d > 0.0 && t >= 0.0 && isfinite(d) && isfinite(t))) {
            s.status = CMC_ST_BAD_CELL;
            atomicOr(status, CMC_ST_BAD_CELL);
        } else {
            const phys::Screen sc = phys::screening(Z, z, d, t);
            s.d = cell_tab<double>(sc, ax);
            s.f = cell_tab<float>(sc, ax);
        }
        W.cs[c] = s;
    }
}

template <typename R>
__device__ __forceinline__ const CellTab<R>& pick(const CellState& s);
template <>
__device__ __forceinline__ const CellTab<double>& pick<double>(const CellState& s) { return s.d; }
template <>
__device__ __forceinline__ const CellTab<float>& pick<float>(const CellState& s) { return s.f; }

// ------------------------------------------------------------------ teams
// A team runs one cell: the whole workgroup (kT = 256) or one wavefront
// (kT = 64: four cells per workgroup and no workgroup barrier at all).
template <int kT>
struct Team {
    static_assert(kT == 64 || kT == 256, "team of one wavefront or one workgroup");
    static __device__ __forceinline__ int tid() { return kT == 64 ? (int)(threadIdx.x & 63u) : (int)threadIdx.x; }
    static __device__ __forceinline__ void sync() {
        if constexpr (kT == 64) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    }
};

// inclusive prefix sum over the team in thread order
template <int kT>
__device__ __forceinline__ uint32_t team_incl_scan(uint32_t v, uint32_t* red) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if constexpr (kT == 64) {
        return v;
    } else {
        const int w = threadIdx.x >> 6;
        if (lane == 63) red[w] = v;
        __syncthreads();
        uint32_t before = 0;
        for (int i = 0; i < w; ++i) before += red[i];
        __syncthreads();
        return v + before;
    }
}

// exclusive scan of n counters in LDS, in place
template <int kT>
__device__ void team_excl_scan(uint32_t* a, int n, uint32_t* red) {
    const int t = Team<kT>::tid();
    const int per = (n + kT - 1) / kT;
    const int lo = t * per, hi = min(n, lo + per);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += a[i];
    uint32_t run = team_incl_scan<kT>(s, red) - s;
    for (int i = lo; i < hi; ++i) { const uint32_t v = a[i]; a[i] = run; run += v; }
    Team<kT>::sync();
}

template <int kT>
__device__ __forceinline__ bool team_any(bool v, int* red) {
    if constexpr (kT == 64) return __ballot(v) != 0ull;
    else return block_or(v, red) != 0;
}

// Sums over i in [0, n) in one fixed order whatever the team size: as 256
// threads striding by 256, each wavefront's partials reduced by wave_sum
// and the four wavefront totals added in order (team_reduce4).
// The two team shapes therefore give bit-identical densities and n_ab.
// canon_part2 is the per-thread part before the cross-wavefront step
// (wavefront teams: the team total); it walks once and accumulates two sums.
// A thread reads four terms at a time (indices clamped into [0, n), so the
// reads are issued together) and then adds those below n in the canonical
// order: each term is first added to zero, which gives it exactly.
template <int kT, typename F>
__device__ __forceinline__ void canon_part2(int n, F f, double& s1, double& s2) {
    if constexpr (kT == 256) {
        double a = 0.0, b = 0.0;
        for (int q = threadIdx.x; q < n; q += 1024) {
            double ta[4], tb[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ta[r] = 0.0; tb[r] = 0.0;
                f(min(q + 256 * r, n - 1), ta[r], tb[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (q + 256 * r < n) { a += ta[r]; b += tb[r]; }
        }
        s1 = wave_sum(a); s2 = wave_sum(b);
    } else {
        const int l = threadIdx.x & 63;
        double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = l; q < n; q += 256) {
            double ta[4], tb[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ta[r] = 0.0; tb[r] = 0.0;
                f(min(q + 64 * r, n - 1), ta[r], tb[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (q + 64 * r < n) { a[r] += ta[r]; b[r] += tb[r]; }
        }
        s1 = ((wave_sum(a[0]) + wave_sum(a[1])) + wave_sum(a[2])) + wave_sum(a[3]);
        s2 = ((wave_sum(b[0]) + wave_sum(b[1])) + wave_sum(b[2])) + wave_sum(b[3]);
    }
}

template <int kT, typename F>
__device__ __forceinline__ double canon_part(int n, F f) {
    double s1, s2;
    canon_part2<kT>(n, [&](int q, double& a, double& b) { a += f(q); }, s1, s2);
    return s1;
}

// the cross-wavefront step of four canonical sums and an OR, one round
template <int kT>
__device__ __forceinline__ void team_reduce4(double (&v)[4], bool& flag, double* red4, int* redi) {
    const bool wf = __ballot(flag) != 0ull;
    if constexpr (kT == 64) {
        flag = wf;
    } else {
        const int w = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red4[w * 4 + k] = v[k];
            redi[w] = wf;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = ((red4[k] + red4[4 + k]) + red4[8 + k]) + red4[12 + k];
        flag = (redi[0] | redi[1] | redi[2] | redi[3]) != 0;
        __syncthreads();
    }
}

// team_reduce4 with a word of flag bits OR-ed over the team (bits 0..2)
template <int kT>
__device__ __forceinline__ void team_reduce4_bits(double (&v)[4], int& bits, double* red4, int* redi) {
    int wb = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b)
        if (__ballot((bits >> b) & 1) != 0ull) wb |= 1 << b;
    if constexpr (kT == 64) {
        bits = wb;
    } else {
        const int w = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red4[w * 4 + k] = v[k];
            redi[w] = wb;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = ((red4[k] + red4[4 + k]) + red4[8 + k]) + red4[12 + k];
        bits = redi[0] | redi[1] | redi[2] | redi[3];
        __syncthreads();
    }
}

// The canonical sum (as canon_part2) of values met four per thread, at
// q = t + kT u for u = 0..3 with n <= 4 kT (zero where q >= n), added as
// they come: canon_add for each u in order, then canon_end gives the
// thread's partial after its wavefront's butterfly (workgroup teams) or
// the team total (wavefront teams).
template <int kT>
__device__ __forceinline__ void canon_add(double& s, double v, int u) {
    if constexpr (kT == 256) s = u == 0 ? v : s + v;
    else s = u == 0 ? wave_sum(v) : s + wave_sum(v);
}
template <int kT>
__device__ __forceinline__ double canon_end(double s) {
    if constexpr (kT == 256) return wave_sum(s);
    else return s;
}

// Buckets of the rank sort: the power of two at or above n (at most 4096),
// so that a bucket holds one or two keys on average.
__host__ __device__ inline int rank_bucket_bits(int n) {
    int b = 4;
    while (b < 12 && (1 << b) < n) ++b;
    return b;
}

// Order of n particles by (Philox key, index).  The keys are counted into
// buckets by their top bits, scattered into bucket order (key and index
// side by side), and each one's rank is its bucket's start plus the number
// of bucket members before it; no result depends on the order of the LDS
// atomics.  The keys are drawn twice (count, scatter) instead of being
// stored.  inverse: out[i] = rank of i; else out[rank] = i.
template <int kT>
__device__ void rank_order(int n, uint32_t cell, uint32_t tag, const Rng& rng, uint32_t* sk,
                           uint16_t* tmp, uint32_t* hist, uint16_t* out, bool inverse, uint32_t* red) {
    const int t = Team<kT>::tid();
    const int bb = rank_bucket_bits(n), nb = 1 << bb, sh = 32 - bb;
    for (int b = t; b < nb; b += kT) hist[b] = 0u;
    Team<kT>::sync();
    const int nq = (n + 3) >> 2;
    for (int q = t; q < nq; q += kT) {
        const U4 r = rng.draw((uint32_t)q, cell, tag);
        const uint32_t w4[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (4 * q + u < n) atomicAdd(&hist[w4[u] >> sh], 1u);
    }
    Team<kT>::sync();
    team_excl_scan<kT>(hist, nb, red);
    for (int q = t; q < nq; q += kT) {
        const U4 r = rng.draw((uint32_t)q, cell, tag);
        const uint32_t w4[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = 4 * q + u;
            if (i < n) {
                const uint32_t pos = atomicAdd(&hist[w4[u] >> sh], 1u);
                sk[pos] = w4[u];
                tmp[pos] = (uint16_t)i;
            }
        }
    }
    Team<kT>::sync();
    // hist[b] is now the end of bucket b
    for (int p = t; p < n; p += kT) {
        const uint32_t k = sk[p];
        const int i = tmp[p];
        const int b = (int)(k >> sh);
        const int lo = b ? (int)hist[b - 1] : 0, hi = (int)hist[b];
        int r = lo;
        for (int m = lo; m < hi; ++m) {
            const uint32_t km = sk[m];
            r += (km < k) | ((km == k) & ((int)tmp[m] < i));
        }
        if (inverse) out[i] = (uint16_t)r; else out[r] = (uint16_t)i;
    }
    Team<kT>::sync();
}

// Particles that pair once more when the mobile species is cycled: the e
// of smallest (key, index) among n <= 4 kT, in the order rank_order forms
// (the key of particle i is word i & 3 of the draw keyed by i >> 2), found
// without forming that order.  The keys are counted by their top 8 bits;
// every key in a bin below the one where the count reaches e is selected,
// and the keys of that bin are ranked among themselves.  Sets the bits of
// the selected particles in sel.  Returns false (nothing decided) when
// that bin holds more than kSelList keys: the caller then forms the order.
// LDS: kSelBytes at scr, the last of them the bitmap sel (32 words).
constexpr int kSelList = 128;
constexpr int kSelBytes = 1024 + 8 * kSelList + 16 + 128;

template <int kT>
__device__ bool select_smallest(int n, int e, uint32_t cell, uint32_t tag, const Rng& rng, unsigned char* scr,
                                uint32_t* sel, int t) {
    uint32_t* hist = reinterpret_cast<uint32_t*>(scr);                 // 256 bins
    uint2* list = reinterpret_cast<uint2*>(scr + 1024);                // (key, particle)
    int* sc = reinterpret_cast<int*>(scr + 1024 + 8 * kSelList);       // bin, still needed, list length
    for (int i = t; i < 256; i += kT) hist[i] = 0u;
    for (int i = t; i < 32; i += kT) sel[i] = 0u;
    if (t == 0) sc[2] = 0;
    // n <= 4 kT: one draw per thread gives the keys of particles 4t .. 4t + 3
    const bool has = 4 * t < n;
    U4 r{0u, 0u, 0u, 0u};
    if (has) r = rng.draw((uint32_t)t, cell, tag);
    const uint32_t k4[4] = {r.x, r.y, r.z, r.w};
    Team<kT>::sync();
    if (has) {
#pragma unroll
        for (int w = 0; w < 4; ++w)
            if (4 * t + w < n) atomicAdd(&hist[k4[w] >> 24], 1u);
    }
    Team<kT>::sync();
    if (t < 64) {
        // the first wavefront finds the bin where the count reaches e
        const uint32_t h[4] = {hist[4 * t], hist[4 * t + 1], hist[4 * t + 2], hist[4 * t + 3]};
        const uint32_t sum = h[0] + h[1] + h[2] + h[3];
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (t >= o) incl += y;
        }
        uint32_t below = incl - sum;
        if (below < (uint32_t)e && (uint32_t)e <= incl) {
            int b = 4 * t + 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (below + h[i] >= (uint32_t)e) { b = 4 * t + i; break; }
                below += h[i];
            }
            sc[0] = b;
            sc[1] = e - (int)below;
        }
    }
    Team<kT>::sync();
    const uint32_t bin = (uint32_t)sc[0];
    if (has) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int p = 4 * t + w;
            if (p >= n) continue;
            const uint32_t top = k4[w] >> 24;
            if (top < bin) {
                atomicOr(&sel[p >> 5], 1u << (p & 31));
            } else if (top == bin) {
                const int slot = atomicAdd(&sc[2], 1);
                if (slot < kSelList) list[slot] = make_uint2(k4[w], (uint32_t)p);
            }
        }
    }
    Team<kT>::sync();
    const int m = sc[2], need = sc[1];
    if (m > kSelList) return false;
    for (int i = t; i < m; i += kT) {
        const uint2 a = list[i];
        int rk = 0;
        for (int j = 0; j < m; ++j) {
            const uint2 o = list[j];
            rk += (o.x < a.x) | ((o.x == a.x) & (o.y < a.y));
        }
        if (rk < need) atomicOr(&sel[a.y >> 5], 1u << (a.y & 31));
    }
    Team<kT>::sync();
    return true;
}

// Pair indices of the open pairs of a pass that formed no order: the rank
// of each one's particle by (key, index) among the n particles of its
// species, counted against every key of the species (drawn again, as
// rank_order draws them).  open[k] = particle | kind << 16; keys[k] gets
// the particle's key, pj[k] its rank.
template <int kT>
__device__ void rank_open(int n, uint32_t cell, uint32_t tag, const Rng& rng, const uint32_t* open,
                          uint32_t* keys, uint32_t* pj, int n_open) {
    const int t = Team<kT>::tid();
    if (t < n_open) {
        const uint32_t m = open[t] & 0xFFFFu;
        const U4 r = rng.draw(m >> 2, cell, tag);
        const uint32_t w4[4] = {r.x, r.y, r.z, r.w};
        keys[t] = w4[m & 3u];
        pj[t] = 0u;
    }
    Team<kT>::sync();
    const int nq = (n + 3) >> 2;
    for (int base = 0; base < nq; base += kT) {
        const int q = base + t;
        uint32_t w4[4] = {0u, 0u, 0u, 0u};
        if (q < nq) {
            const U4 r = rng.draw((uint32_t)q, cell, tag);
            w4[0] = r.x; w4[1] = r.y; w4[2] = r.z; w4[3] = r.w;
        }
        for (int k = 0; k < n_open; ++k) {
            const uint32_t kk = keys[k], mk = open[k] & 0xFFFFu;
            int below = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = 4u * (uint32_t)q + (uint32_t)u;
                const bool lt = q < nq && (int)i < n && (w4[u] < kk || (w4[u] == kk && i < mk));
                below += __popcll(__ballot(lt));
            }
            if ((threadIdx.x & 63u) == 0u) atomicAdd(&pj[k], (uint32_t)below);
        }
    }
    Team<kT>::sync();
}

// j mod n for j < 2^15, n <= 2^14 from a float reciprocal (the quotient is
// off by at most one; checked for every such j and n)
__device__ __forceinline__ int mod_small(int j, int n, float rn) {
    int r = j - (int)((float)j * rn) * n;
    r += r < 0 ? n : 0;
    r -= r >= n ? n : 0;
    return r;
}

// per-team LDS of the pass kernel
constexpr int kSliceMax = 168;   // >= kSliceBrems, kSliceBH
// the stream kernel: electrons per cell it takes at most, records in flight
// per thread, threads per cell, wavefronts per SIMD (the second launch
// bound; measured on the foil cells: four with 128 registers beat five or
// six, which spill in the cell's prologue, and more records in flight
// gained nothing)
constexpr int kStreamCap = 4096;
constexpr int kStreamDepth = 2;
constexpr int kStreamThreads = 256;
constexpr int kStreamWaves = 4;

// The team's region holds the arrays of the rank sort or, in the direct
// form of a cycled mobile species, the selection scratch (kSelBytes); the
// table slice follows it.
__host__ __device__ inline size_t team_region(int cap, int kT) {
    (void)kT;
    const size_t n = (size_t)((cap + 63) / 64 * 64);
    const size_t sort = n * 10 + ((size_t)4 << rank_bucket_bits(cap));
    return sort > (size_t)kSelBytes ? sort : (size_t)kSelBytes;
}

__host__ __device__ inline size_t team_bytes(int cap, int rbytes, int kT) {
    return team_region(cap, kT) + (size_t)kSliceMax * rbytes + 16;
}

struct TeamMem {
    uint32_t* keys;   // keys in bucket order
    uint16_t* tmp;    // particle of each bucket slot
    uint32_t* hist;
    uint16_t* ordM;   // mobile species: rank of each particle, or particle of each rank
    uint16_t* ordI;   // ions: particle of each rank
    unsigned char* base;   // the region (selection scratch in the direct form)
    unsigned char* slice;
};

__device__ __forceinline__ TeamMem carve_team(unsigned char* p, int cap, int kT) {
    const size_t n = (size_t)((cap + 63) / 64 * 64);
    TeamMem m;
    m.base = p;
    m.slice = p + team_region(cap, kT);
    m.keys = reinterpret_cast<uint32_t*>(p); p += n * 4;
    m.tmp = reinterpret_cast<uint16_t*>(p); p += n * 2;
    m.hist = reinterpret_cast<uint32_t*>(p); p += (size_t)4 << rank_bucket_bits(cap);
    m.ordM = reinterpret_cast<uint16_t*>(p); p += n * 2;
    m.ordI = reinterpret_cast<uint16_t*>(p);
    return m;
}

// one test settled with P = -expm1(-x) in FP64: the near-threshold count,
// then the event iff U1 < P and U2 < P_ej
// The pass kernels' bound test of a pair, in FP32.  It passes every pair
// whose exact test could hold (an event needs U1 < P, the near band
// U1 <= (1 + near_rel) P, and P = 1 - exp(-x) <= x): the top 24 bits of the
// draw's first word are at most 2^24 U1, and xs, 2^24 rej x formed from a few
// FP32 roundings, stays far above 2^24 (1 + near_rel) x since rej is twice
// 1 + near_rel.  The event kernel settles the pairs it passes in FP64 and
// applies the FP64 bound again.
__device__ __forceinline__ bool bound24(uint32_t rx, float xs) { return (float)(rx >> 8) <= xs; }

__device__ __forceinline__ bool settle(double x, const Rng& rng, uint32_t dk, uint32_t cell, uint32_t tag,
                                       uint32_t tag_hi, double rej, double near_rel, double Pej, int& near) {
    double U1, U2;
    accept_uniforms(rng, dk, cell, tag, tag_hi, U1, U2);
    if (!(U1 <= rej * x)) return false;
    const double P = -expm1(-x);
    if (fabs(U1 - P) <= near_rel * P) near++;
    return U1 < P && U2 < Pej;
}

// list a cell (once) for the event kernel
__device__ __forceinline__ void list_cell(const Work& W, int64_t c) {
    if (!(atomicOr(&W.flags[c], kFlagListed) & kFlagListed)) W.list_ev[atomicAdd(&W.counters[kCntEv], 1)] = (int32_t)c;
}

// a cell the event kernel runs with the sequential step
__device__ __forceinline__ void mark_slow(const Work& W, int64_t c) {
    atomicOr(&W.flags[c], kFlagSlow);
    list_cell(W, c);
}

// a pair the bound on P left open, for the event kernel (beyond kCandCap
// the cell takes the sequential step)
__device__ __forceinline__ void push_cand(const Work& W, int64_t c, uint64_t rec) {
    const int k = atomicAdd(&W.ncand[c], 1);
    if (k == 0) list_cell(W, c);
    if (k < kCandCap) W.cand[c * kCandCap + k] = rec;
    else mark_slow(W, c);
}

// LDS of a team beside its dynamic region: reduction scratch and the open
// pairs found without an order
struct PassLds {
    double* red4;
    uint32_t* redu;
    int* redi;
    uint32_t* opn;      // open pairs found without the order
    uint32_t* opk;      // their particles' keys
    uint32_t* opj;      // their pair indices
    int* nopen;
};

// What the electron-ion pass of a cell hands to the photon-ion pass of the
// same cell when one team runs both: the weight checks passed and whether
// the ions share one weight (flags), and the ions' weight sum.
struct PassCarry {
    int32_t flags;
    double ionsum;
};

// The pass kPass over cell c by one team (see k_pass).  kFused: the same
// team has just run the electron-ion pass of this cell, whose results are
// in carry; otherwise the photon-ion pass reads them from the workspace.
template <typename R, int kT, int kPass, bool kMov, bool kFused>
__device__ __forceinline__ void pass_cell(const StepArgs& A, const TabView<R>& T, const Work& W, int cap, int filter,
                                          int fcap, int slow_cap, int64_t c, const TeamMem M, const Rng rng,
                                          double rej, int t, const PassLds L, PassCarry& carry) {
    R* slice = reinterpret_cast<R*>(M.slice);
    // the cell's parameters in one round of loads: its state, the
    // offsets and live counts of the three species, its global index
    const uint32_t cell = cell_word(A.cid, c);
    const int32_t cstat = W.cs[c].status;
    const int32_t cflags = (kPass == 0 || !kFused) ? W.flags[c] : carry.flags;
    const CellTab<R> ct_c = pick<R>(W.cs[c]);
    const int64_t eo0 = A.el.off[c], eo1 = A.el.off[c + 1], go0 = A.ph.off[c], go1 = A.ph.off[c + 1];
    const int64_t io0 = A.io.off[c], io1 = A.io.off[c + 1];
    const int ecn = A.el.count ? A.el.count[c] : 0x7FFFFFFF, gcn = A.ph.count ? A.ph.count[c] : 0x7FFFFFFF;
    const int icn = A.io.count ? A.io.count[c] : 0x7FFFFFFF;
    if (cstat) return;                                // invalid cell (flagged by k_cell_state)
    if (kPass == 0 && (cflags & kFlagDone0)) {
        // done by the stream kernel, whose results the photon-ion pass takes
        carry = PassCarry{cflags & (kFlagWeightsOk | kFlagIonsSame | kFlagDone1), W.ionsum[c]};
        return;
    }
    if (kPass == 1 && (cflags & kFlagDone1)) return;
    const int Ne = max(0, min(ecn, (int)(eo1 - eo0))), Ng = max(0, min(gcn, (int)(go1 - go0)));
    const int Ni = max(0, min(icn, (int)(io1 - io0)));
    // size classes of the hybrid schedule: filter 1 takes the cells up
    // to fcap particles per species, filter 2 the larger ones
    const int mx = max(Ne, max(Ng, Ni));
    if ((filter == 1 && mx > fcap) || (filter == 2 && mx <= fcap)) return;
    if (Ne > A.maxn || Ng > A.maxn || Ni > A.maxn) {
        if (t == 0) atomicOr(A.status, CMC_ST_TOO_LARGE);
        return;
    }
    const bool ei = (A.proc & (CMC_BREMS | CMC_TRIDENT)) && Ne > 0 && Ni > 0;
    const bool gi = (A.proc & CMC_BH) && Ng > 0 && Ni > 0;
    // cells beyond the largest LDS of the step's pass launches go to the
    // sequential kernel whole
    if ((ei && (Ne > slow_cap || Ni > slow_cap)) || (gi && (Ng > slow_cap || Ni > slow_cap))) {
        if (t == 0) mark_slow(W, c);
        return;
    }
    // every order this pass might need fits this launch's LDS
    const bool fits = kPass == 0 ? (Ne <= cap && Ni <= cap) : (Ng <= cap && Ni <= cap);
    const int64_t e0 = eo0, g0 = go0, i0 = io0;
    const bool active = kPass == 0 ? ei : gi;
    const int Nm = kPass == 0 ? Ne : Ng, No = kPass == 0 ? Ng : Ne;
    const int64_t m0 = kPass == 0 ? e0 : g0;
    const SpeciesDev& S = kPass == 0 ? A.el : A.ph;
    const double* wm = S.w + m0;
    const double* wo = kPass == 0 ? A.ph.w + g0 : A.el.w + e0;
    const double* wion = A.io.w + i0;
    const bool mobA = Nm >= Ni;
    const int N = mobA ? Nm : Ni;
    // ---- direct form: ions at rest, at most four mobile particles per
    // thread.  The weights are summed (densities, the mobile particles'
    // n_ab terms against the first ion's weight, the weight checks) in
    // one reduction, beside the table slice; then every pair is tested
    // in storage order of its mobile particle.  A cycled mobile species
    // (N_m < N_i, K = N_i div N_m pairs per particle, e = N_i mod N_m of
    // them one more) takes the e particles of smallest key as the order
    // would, found by select_smallest; n_ab = fma(K, A, B), A the
    // canonical sum of the terms and B that of the selected particles'.
    // Should the ions not share one weight, the cell is done again below
    // with both orders.
    if constexpr (!kMov) {
        if (active && fits && N <= 4 * kT) {
            const bool cyc = !mobA;
            const int K = N / Nm, e = N - K * Nm;
            uint32_t* sel = reinterpret_cast<uint32_t*>(M.base + kSelBytes - 128);
            {
                const CellTab<R> ct = ct_c;
                if (kPass == 0) {
                    if (A.proc & CMC_BREMS)
                        for (int i = t; i < kSliceBrems; i += kT) slice[i] = slice_node_brems<R>(T, ct, i);
                } else {
                    for (int i = t; i < kSliceBH; i += kT) slice[i] = slice_node_bh<R>(T, ct, i);
                }
            }
            // the first pair's momenta are in flight during the reduction
            double nx = 0.0, ny = 0.0, nz = 0.0;
            if (t < Nm) { nx = S.px[m0 + t]; ny = S.py[m0 + t]; nz = S.pz[m0 + t]; }
            const double w0 = wion[0];
            int fl = 0;                 // 1 bad weight, 2 ions of unequal weight, 4 above the tables
            double v4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = t + kT * u;
                const double wq = q < Nm ? wm[q] : 0.0, wi = q < Ni ? wion[q] : 0.0;
                fl |= (!(wq >= 0.0) || !isfinite(wq) || !(wi >= 0.0) || !isfinite(wi)) ? 1 : 0;
                fl |= (q < Ni && wi != w0) ? 2 : 0;
                canon_add<kT>(v4[0], wq, u);
                canon_add<kT>(v4[1], q < Nm ? (wq < w0 ? wq : w0) : 0.0, u);
                canon_add<kT>(v4[2], wi, u);
            }
            v4[0] = canon_end<kT>(v4[0]);
            v4[1] = canon_end<kT>(v4[1]);
            v4[2] = canon_end<kT>(v4[2]);
            {
                int bad = 0;
                v4[3] = canon_part<kT>(No, [&](int q) { const double w = wo[q]; bad |= !(w >= 0.0) || !isfinite(w); return w; });
                fl |= bad ? 1 : 0;
            }
            if (t == 0) L.nopen[0] = 0;
            team_reduce4_bits<kT>(v4, fl, L.red4, L.redi);   // its barriers also publish the slice
            if (kT == 64) Team<kT>::sync();
            if (kPass == 0 && !(fl & 1) && t == 0) {
                W.ionsum[c] = v4[2];
                atomicOr(&W.flags[c], kFlagWeightsOk | ((fl & 2) ? 0 : kFlagIonsSame));
            }
            if (kPass == 0 && !(fl & 1)) carry = PassCarry{kFlagWeightsOk | ((fl & 2) ? 0 : kFlagIonsSame), v4[2]};
            bool chosen = true;
            if (!(fl & 3) && cyc) {
                // indices of the cycled case come from an opaque copy of the
                // thread's index: formed here, not kept across cells in
                // registers that the pairs need
                int tt = t;
                asm volatile("" : "+v"(tt));
                if (e > 0)
                    chosen = select_smallest<kT>(Nm, e, cell, kPass == 0 ? kTagKeyE : kTagKeyG, rng, M.base, sel, tt);
                if (chosen) {
                    double vb[4] = {0.0, 0.0, 0.0, 0.0};
                    if (e > 0) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int q = tt + kT * u;
                            const bool sq = q < Nm && ((sel[q >> 5] >> (q & 31)) & 1u);
                            const double wq = sq ? wm[q] : 0.0;
                            canon_add<kT>(vb[0], sq ? (wq < w0 ? wq : w0) : 0.0, u);
                        }
                        vb[0] = canon_end<kT>(vb[0]);
                        bool none = false;
                        team_reduce4<kT>(vb, none, L.red4, L.redi);
                    }
                    v4[1] = fma((double)K, v4[1], vb[0]);   // one rounding, as in the ordered form
                }
            }
            if (!(fl & 2) && chosen) {
                if (fl & 1) {
                    if (t == 0) atomicOr(A.status, CMC_ST_BAD_WEIGHT);
                    return;
                }
                const double nab = v4[1];
                int high = 0;
                if (nab > 0.0) {
                    const double coef = v4[0] * v4[2] / nab;
                    const float kx = (float)(coef * A.dt * rej * 16777216.0);
                    // workgroup teams: the first pairs of a thread's particles
                    // q = t + 256 u share the draw of the upper bits of U1
                    // (hi_group(q) = t, word u), drawn once per process
                    const uint32_t tagA = kPass == 0 ? kTagHiBr : kTagHiBh;
                    U4 hA{0u, 0u, 0u, 0u}, hT{0u, 0u, 0u, 0u};
                    if constexpr (kT == 256) {
                        if (kPass == 1 || (A.proc & CMC_BREMS)) hA = rng.draw(hi_group((uint32_t)t), cell, tagA);
                        if (kPass == 0 && (A.proc & CMC_TRIDENT)) hT = rng.draw(hi_group((uint32_t)t), cell, kTagHiTr);
                    }
                    // the word of U1's upper bits for the pair keyed by x:
                    // the shared one for a particle's first pair
                    const auto word = [&](uint32_t x, bool first, uint32_t shared, uint32_t tag) {
                        return kT == 256 && first ? shared : hi_word(rng.draw(hi_group(x), cell, tag), (x >> 8) & 3u);
                    };
                    // every particle's first pair, one at a time (the tests do
                    // not overlap in registers), the next momenta in flight
#pragma unroll 1
                    for (int u = 0; u < 4; ++u) {
                        const int q = t + kT * u;
                        const double cx = nx, cy = ny, cz = nz;
                        if (q + kT < Nm) { nx = S.px[m0 + q + kT]; ny = S.py[m0 + q + kT]; nz = S.pz[m0 + q + kT]; }
                        // word u of the shared draws: the words move down one per pair
                        const uint32_t wA = hA.x, wT = hT.x;
                        hA = U4{hA.y, hA.z, hA.w, 0u};
                        hT = U4{hT.y, hT.z, hT.w, 0u};
                        if (q >= Nm) continue;
                        uint32_t bits = 0;
                        if (kPass == 0) {
                            const Elec<R> el = electron_p<R>(cx, cy, cz);
                            if (A.proc & CMC_BREMS) {
                                bool hi;
                                const R sig = brems_sig_slice<R>(T, slice, el.g, el.gm1, hi);
                                high |= hi;
                                if (sig > (R)0 && bound24(word((uint32_t)q, true, wA, kTagHiBr), kx * (float)sig * (float)el.vrel))
                                    bits = 1u;
                            }
                            if ((A.proc & CMC_TRIDENT) && !bits) {
                                const R sig = (R)phys::trident_sigma(T.Z, (double)el.g);
                                if (sig > (R)0 && bound24(word((uint32_t)q, true, wT, kTagHiTr), kx * (float)sig * (float)el.vrel))
                                    bits = 2u;
                            }
                        } else {
                            bool hi;
                            const R sig = bh_sig_slice<R>(T, slice, photon_k<R>(cx, cy, cz), hi);
                            high |= hi;
                            if (sig > (R)0 && bound24(word((uint32_t)q, true, wA, kTagHiBh), kx * (float)sig * (float)phys::kC))
                                bits = 1u;
                        }
                        if (bits) {
                            const int o = atomicAdd(&L.nopen[0], 1);
                            if (o < kCandCap) L.opn[o] = (uint32_t)q | (bits << 16);
                        }
                    }
                    // cycled mobile species: the further pairs k = 1 .. reps - 1 of
                    // each particle (K - 1 for all, one more for the selected),
                    // keyed by q + k N_m, the momenta read again
                    if (cyc && (K > 1 || e > 0)) {
                        int tt = t;
                        asm volatile("" : "+v"(tt));
#pragma unroll 1
                        for (int u = 0; u < 4; ++u) {
                            const int q = tt + kT * u;
                            if (q >= Nm) continue;
                            const int reps = K + ((e > 0 && ((sel[q >> 5] >> (q & 31)) & 1u)) ? 1 : 0);
                            if (reps < 2) continue;
                            const double cx = S.px[m0 + q], cy = S.py[m0 + q], cz = S.pz[m0 + q];
                            for (int k = 1; k < reps; ++k) {
                                const uint32_t x = (uint32_t)(q + k * Nm);
                                uint32_t bits = 0;
                                if (kPass == 0) {
                                    const Elec<R> el = electron_p<R>(cx, cy, cz);
                                    bool hi;
                                    const R sb = (A.proc & CMC_BREMS) ? brems_sig_slice<R>(T, slice, el.g, el.gm1, hi) : (R)0;
                                    if (sb > (R)0 && bound24(word(x, false, 0u, kTagHiBr), kx * (float)sb * (float)el.vrel))
                                        bits = 1u;
                                    const R st = (A.proc & CMC_TRIDENT) ? (R)phys::trident_sigma(T.Z, (double)el.g) : (R)0;
                                    if (!bits && st > (R)0 && bound24(word(x, false, 0u, kTagHiTr), kx * (float)st * (float)el.vrel))
                                        bits = 2u;
                                } else {
                                    bool hi;
                                    const R sig = bh_sig_slice<R>(T, slice, photon_k<R>(cx, cy, cz), hi);
                                    if (sig > (R)0 && bound24(word(x, false, 0u, kTagHiBh), kx * (float)sig * (float)phys::kC))
                                        bits = 1u;
                                }
                                if (bits) {
                                    const int o = atomicAdd(&L.nopen[0], 1);
                                    if (o < kCandCap) L.opn[o] = (uint32_t)q | (bits << 16) | ((uint32_t)k << 20);
                                }
                            }
                        }
                    }
                    Team<kT>::sync();
                    const int n_open = L.nopen[0];
                    if (n_open > kCandCap) {
                        if (t == 0) mark_slow(W, c);
                    } else if (n_open > 0) {
                        // pair index of an open pair: its particle's rank plus k N_m
                        rank_open<kT>(Nm, cell, kPass == 0 ? kTagKeyE : kTagKeyG, rng, L.opn, L.opk, L.opj, n_open);
                        if (t < n_open) {
                            const uint32_t o = L.opn[t];
                            push_cand(W, c, ev_pack(kPass, (int)L.opj[t] + (int)(o >> 20) * Nm, (int)(o & 0xFFFFu), 0,
                                                    (o >> 16) & 0xFu));
                        }
                    }
                    if (t == 0) W.coef[c * 2 + kPass] = coef;
                }
                if (t == 0) {
                    if (kPass == 0) {
                        A.ti[c * CMC_NI + CMC_I_PAIRS_BR] = (nab > 0.0 && (A.proc & CMC_BREMS)) ? N : 0;
                        A.ti[c * CMC_NI + CMC_I_PAIRS_TR] = (nab > 0.0 && (A.proc & CMC_TRIDENT)) ? N : 0;
                        A.td[c * CMC_ND + CMC_D_NAB_EI] = nab;
                    } else {
                        A.ti[c * CMC_NI + CMC_I_PAIRS_BH] = nab > 0.0 ? N : 0;
                        A.td[c * CMC_ND + CMC_D_NAB_GI] = nab;
                    }
                }
                if (team_any<kT>(high != 0, L.redi) && t == 0) atomicOr(A.status, CMC_ST_GAMMA_HIGH);
                Team<kT>::sync();   // LDS of this cell is free
                return;
            }
            Team<kT>::sync();       // the slice is staged again below
        }
    }
    // the weights of the cell are checked (non-negative, finite) as
    // they are summed into the densities
    int bad = 0;
    const auto chk = [&bad](double v) { bad |= !(v >= 0.0) || !isfinite(v); return v; };
    double v4[4];   // n_mobile, n_ab, n_ion, n_other
    // When the cell's ions are at rest and share one weight, no decision
    // and no product depends on which ion a pair gets (P_ej and n_ab see
    // only that weight): the ion order is then not formed, and the open
    // pairs name ion 0.
    const double wi0 = Ni > 0 ? wion[0] : 0.0;
    // after the electron-ion pass of this step (photon-ion pass): the ion
    // sum, the ions' sameness and every weight check are known
    const bool known = kPass == 1 && (cflags & kFlagWeightsOk);
    bool same = true;
    if (known) {
        // the team reduction below adds the wavefronts' partials: the
        // total enters through the first wavefront alone
        v4[2] = (kT == 64 || threadIdx.x < 64) ? (kFused ? carry.ionsum : W.ionsum[c]) : 0.0;
        same = (cflags & kFlagIonsSame) != 0;
    } else {
        v4[2] = canon_part<kT>(Ni, [&](int q) { const double w = wion[q]; same &= w == wi0; return chk(w); });
    }
    const bool uneq = team_any<kT>(!same, L.redi);
    const bool ion_order = active && (kMov || uneq);
    // When every mobile particle pairs once, the draws of a pair are
    // keyed by its mobile particle: with interchangeable ions nothing
    // then depends on the order, which is not formed; the few open pairs
    // get their pair index (the rank of their particle) at the end.
    const bool mob_order = active && (!mobA || ion_order);
    // a cycled mobile species against interchangeable ions: its tests are
    // walked by draw group (below)
    const bool cyc_fast = active && !mobA && !ion_order;
    if (active && !fits && ((ion_order && Ni > cap) || (mob_order && Nm > cap))) {
        // an order larger than this launch's LDS: the large-LDS launch takes
        // the pass (listed once per step, however often the launch runs)
        const int32_t fb = kPass == 0 ? kFlagBig0 : kFlagBig1;
        if (t == 0 && !(atomicOr(&W.flags[c], fb) & fb))
            W.list_big[kPass][atomicAdd(&W.counters[kPass == 0 ? kCntBig0 : kCntBig1], 1)] = (int32_t)c;
        return;
    }
    if (t == 0) L.nopen[0] = 0;
    // when every mobile particle pairs once the pair loop walks them in
    // storage order: its first momenta are loaded before the sort
    double qx = 0.0, qy = 0.0, qz = 0.0;
    if (active) {
        if (mobA && t < N) { qx = S.px[m0 + t]; qy = S.py[m0 + t]; qz = S.pz[m0 + t]; }
        const CellTab<R> ct = pick<R>(W.cs[c]);
        if (kPass == 0) {
            if (A.proc & CMC_BREMS)
                for (int i = t; i < kSliceBrems; i += kT) slice[i] = slice_node_brems<R>(T, ct, i);
        } else {
            for (int i = t; i < kSliceBH; i += kT) slice[i] = slice_node_bh<R>(T, ct, i);
        }
        if (mob_order)
            rank_order<kT>(Nm, cell, kPass == 0 ? kTagKeyE : kTagKeyG, rng, M.keys, M.tmp, M.hist, M.ordM, mobA, L.redu);
        else
            Team<kT>::sync();      // the slice and the open-pair count
        if (ion_order)
            rank_order<kT>(Ni, cell, kPass == 0 ? kTagKeyIE : kTagKeyIG, rng, M.keys, M.tmp, M.hist, M.ordI, false, L.redu);
    }
    const float rNm = 1.0f / (float)Nm, rNi = 1.0f / (float)Ni;
    // the smaller species is cycled (j mod N_B); the other one is not
    const auto ion_of = [&](int j) { return ion_order ? (int)M.ordI[Ni == N ? j : mod_small(j, Ni, rNi)] : 0; };
    const auto w_ion = [&](int j) { return ion_order ? wion[ion_of(j)] : wi0; };
    const auto mob_of = [&](int j) { return (int)M.ordM[Nm == N ? j : mod_small(j, Nm, rNm)]; };
    // a cycled mobile species is walked in rank order: its first momenta
    // are read once the order is formed
    if (active && !mobA && !cyc_fast && t < N) { const int m = mob_of(t); qx = S.px[m0 + m]; qy = S.py[m0 + m]; qz = S.pz[m0 + m]; }
    // the other weights, read once: the densities n = sum W, n_ab =
    // sum_j min(W_a, W_b) and the weight check (when every mobile
    // particle pairs once, its density and n_ab share the walk)
    double cyc_b = 0.0;
    int cyc_k = 0;
    if (active && mobA) {
        canon_part2<kT>(N, [&](int q, double& a, double& b) {
            const double u = chk(wm[q]), v = ion_order ? w_ion((int)M.ordM[q]) : wi0;
            a += u;
            b += u < v ? u : v;
        }, v4[0], v4[1]);
    } else if (active && !ion_order) {
        // a cycled mobile species with interchangeable ions: n_ab = K A + B
        // as the direct form forms it (A over all the mobile particles' terms,
        // B over those of the e particles of smallest key, ranks 0 .. e - 1)
        uint32_t* selb = reinterpret_cast<uint32_t*>(M.hist);   // free once the order is formed
        for (int i = t; i < (Nm + 31) / 32; i += kT) selb[i] = 0u;
        Team<kT>::sync();
        for (int r = t; r < N - (N / Nm) * Nm; r += kT) {
            const int p = (int)M.ordM[r];
            atomicOr(&selb[p >> 5], 1u << (p & 31));
        }
        Team<kT>::sync();
        canon_part2<kT>(Nm, [&](int q, double& a, double& b) {
            const double u = chk(wm[q]);
            a += u;
            b += u < wi0 ? u : wi0;
        }, v4[0], v4[1]);
        cyc_b = canon_part<kT>(Nm, [&](int q) {
            const double u = wm[q];
            return ((selb[q >> 5] >> (q & 31)) & 1u) ? (u < wi0 ? u : wi0) : 0.0;
        });
        cyc_k = N / Nm;
    } else {
        v4[0] = canon_part<kT>(Nm, [&](int q) { return chk(wm[q]); });
        v4[1] = !active ? 0.0 : canon_part<kT>(N, [&](int j) {
            const double u = wm[mob_of(j)], v = w_ion(j);
            return u < v ? u : v;
        });
    }
    v4[3] = known ? 0.0 : canon_part<kT>(No, [&](int q) { return chk(wo[q]); });
    bool badw = bad != 0;
    team_reduce4<kT>(v4, badw, L.red4, L.redi);
    if (kPass == 0 && !badw && t == 0) {
        W.ionsum[c] = v4[2];
        atomicOr(&W.flags[c], kFlagWeightsOk | (uneq ? 0 : kFlagIonsSame));
    }
    if (kPass == 0 && !badw) carry = PassCarry{kFlagWeightsOk | (uneq ? 0 : kFlagIonsSame), v4[2]};
    if (cyc_k > 0) {
        double vb[4] = {cyc_b, 0.0, 0.0, 0.0};
        bool none = false;
        team_reduce4<kT>(vb, none, L.red4, L.redi);
        v4[1] = fma((double)cyc_k, v4[1], vb[0]);   // one rounding, as in the direct form
    }
    if (badw) {
        if (t == 0) atomicOr(A.status, CMC_ST_BAD_WEIGHT);
        return;
    }
    if (!active) return;
    const double nab = v4[1];
    int high = 0;
    if (nab > 0.0) {
        const double coef = v4[0] * v4[2] / nab;
        const float kx = (float)(coef * A.dt * rej * 16777216.0);
        // the draw holding U1's upper bits serves the four pairs of its
        // group (keys x, x + 256, x + 512, x + 768): the last one drawn is
        // kept per process, so a workgroup thread walking its mobile
        // particles in storage order (q = t + 256 u) draws once per four
        uint32_t g_br = 0xFFFFFFFFu, g_tr = 0xFFFFFFFFu;
        U4 h_br{0u, 0u, 0u, 0u}, h_tr{0u, 0u, 0u, 0u};
        const auto hi_bits = [&](uint32_t x, uint32_t tag, uint32_t& gk, U4& h) {
            const uint32_t gx = hi_group(x);
            if (gx != gk) { h = rng.draw(gx, cell, tag); gk = gx; }
            return hi_word(h, (x >> 8) & 3u);
        };
        if (cyc_fast) {
            // N = N_ion pairs: particle m of the cycled species pairs K = N div
            // N_m times and, if its rank is below e = N mod N_m, once more
            // (Sec. III.A pairing).  All its tests share one cross section and
            // flux: its bounds are formed once (in the arithmetic of the tests
            // below the other forms make), and the tests are walked by draw
            // group: the keys x = m + k N_m of a group ((x >> 10) << 8 |
            // (x & 255) = g) are base(g) + 256 w, w = 0..3, and share the draw
            // of U1's upper bits, word w.
            // LDS of the team (n >= N_m entries each): the bounds in the key
            // array and over the two order arrays (4 n bytes, written once
            // the ranks are taken from the order), the ranks in the bucket
            // particle array, the selection bitmap in the histogram
            float* xb = reinterpret_cast<float*>(M.keys);   // first process's bound of m (< 0: none)
            float* xt = reinterpret_cast<float*>(M.ordM);   // Trident's bound of m (over ordM, ordI)
            uint16_t* rk = M.tmp;                           // rank of m
            const uint32_t* selb = reinterpret_cast<const uint32_t*>(M.hist);
            for (int r = t; r < Nm; r += kT) rk[M.ordM[r]] = (uint16_t)r;
            Team<kT>::sync();
            for (int m = t; m < Nm; m += kT) {
                const double cx = S.px[m0 + m], cy = S.py[m0 + m], cz = S.pz[m0 + m];
                float b1 = -1.0f, b2 = -1.0f;
                if (kPass == 0) {
                    const Elec<R> e = electron_p<R>(cx, cy, cz);
                    if (A.proc & CMC_BREMS) {
                        bool hi;
                        const R sig = brems_sig_slice<R>(T, slice, e.g, e.gm1, hi);
                        high |= hi;
                        if (sig > (R)0) b1 = kx * (float)sig * (float)e.vrel;
                    }
                    if (A.proc & CMC_TRIDENT) {
                        const R sig = (R)phys::trident_sigma(T.Z, (double)e.g);
                        if (sig > (R)0) b2 = kx * (float)sig * (float)e.vrel;
                    }
                } else {
                    bool hi;
                    const R sig = bh_sig_slice<R>(T, slice, photon_k<R>(cx, cy, cz), hi);
                    high |= hi;
                    if (sig > (R)0) b1 = kx * (float)sig * (float)phys::kC;
                }
                xb[m] = b1;
                xt[m] = b2;
            }
            Team<kT>::sync();
            const int K = N / Nm, e = N - K * Nm;
            const int X = K * Nm + (e > 0 ? Nm : 0);      // keys of every particle's last pair and below
            const int G = ((X + 1023) >> 10) << 8;
            for (int g = t; g < G; g += kT) {
                const int base = ((g >> 8) << 10) | (g & 255);
                if (base >= X) continue;
                const U4 h = rng.draw((uint32_t)g, cell, kPass == 0 ? kTagHiBr : kTagHiBh);
                U4 h2{0u, 0u, 0u, 0u};
                bool h2_drawn = false;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int x = base + 256 * w;
                    if (x >= X) break;
                    const int m = mod_small(x, Nm, rNm);
                    const int k = __float2int_rn((float)(x - m) * rNm);
                    if (!(k < K || ((selb[m >> 5] >> (m & 31)) & 1u))) continue;
                    uint32_t bits = 0;
                    if (bound24(hi_word(h, (uint32_t)w), xb[m])) {
                        bits = 1u;
                    } else if (kPass == 0 && xt[m] >= 0.0f) {
                        if (!h2_drawn) { h2 = rng.draw((uint32_t)g, cell, kTagHiTr); h2_drawn = true; }
                        if (bound24(hi_word(h2, (uint32_t)w), xt[m])) bits = 2u;
                    }
                    if (bits) {
                        const int o = atomicAdd(&L.nopen[0], 1);
                        if (o < kCandCap) L.opn[o] = (uint32_t)m | (bits << 14) | ((uint32_t)k << 16);
                    }
                }
            }
            Team<kT>::sync();
            const int n_open = L.nopen[0];
            if (n_open > kCandCap) {
                if (t == 0) mark_slow(W, c);
            } else if (t < n_open) {
                // pair index: the particle's rank plus k N_m
                const uint32_t o = L.opn[t];
                const int m = (int)(o & 0x3FFFu), k = (int)(o >> 16);
                push_cand(W, c, ev_pack(kPass, (int)rk[m] + k * Nm, m, 0, (o >> 14) & 3u));
            }
        } else {
        for (int q = t; q < N; q += kT) {
            const int j = mobA ? (mob_order ? (int)M.ordM[q] : 0) : q;
            const int jm = mobA ? 0 : (Nm == N ? j : mod_small(j, Nm, rNm));   // rank of the cycled particle
            const int mi = mobA ? q : (int)M.ordM[jm];
            // counter of the pair's draws: its mobile particle and repetition
            const uint32_t dk = (uint32_t)(mobA ? mi : mi + (j - jm));
            // this pair's momenta; the next pair's are read meanwhile
            const double cx = qx, cy = qy, cz = qz;
            if (q + kT < N) {
                const int mn = mobA ? q + kT : mob_of(q + kT);
                qx = S.px[m0 + mn]; qy = S.py[m0 + mn]; qz = S.pz[m0 + mn];
            }
            uint32_t bits = 0;
            Ion b{0.0, 0.0, 0.0, 1.0, false};
            if constexpr (kMov) b = ion_at(A.io, i0 + ion_of(j));
            if (kPass == 0) {
                Elec<R> e;
                if constexpr (kMov) e = electron_moving<R>(electron_frame(b, cx, cy, cz), b);
                else e = electron_p<R>(cx, cy, cz);
                if (A.proc & CMC_BREMS) {
                    bool hi;
                    const R sig = brems_sig_slice<R>(T, slice, e.g, e.gm1, hi);
                    high |= hi;
                    if (sig > (R)0 && bound24(hi_bits(dk, kTagHiBr, g_br, h_br), kx * (float)sig * (float)e.vrel))
                        bits = 1u;
                }
                if ((A.proc & CMC_TRIDENT) && !bits) {
                    const R sig = (R)phys::trident_sigma(T.Z, (double)e.g);
                    if (sig > (R)0 && bound24(hi_bits(dk, kTagHiTr, g_tr, h_tr), kx * (float)sig * (float)e.vrel))
                        bits = 2u;
                }
            } else {
                R k;
                double flux = phys::kC;
                if constexpr (kMov) {
                    const Frame f = photon_frame(b, cx, cy, cz);
                    k = (R)f.g;
                    flux = photon_flux(f, b);
                } else {
                    k = photon_k<R>(cx, cy, cz);
                }
                bool hi;
                const R sig = bh_sig_slice<R>(T, slice, k, hi);
                high |= hi;
                if (sig > (R)0 && bound24(hi_bits(dk, kTagHiBh, g_br, h_br), kx * (float)sig * (float)flux))
                    bits = 1u;
            }
            if (bits) {
                if (mob_order) {
                    push_cand(W, c, ev_pack(kPass, j, mi, ion_of(j), bits));
                } else {
                    const int k = atomicAdd(&L.nopen[0], 1);
                    if (k < kCandCap) L.opn[k] = (uint32_t)mi | (bits << 16);
                }
            }
        }
        if (!mob_order) {
            Team<kT>::sync();
            const int n_open = L.nopen[0];
            if (n_open > kCandCap) {
                if (t == 0) mark_slow(W, c);
            } else if (n_open > 0) {
                rank_open<kT>(Nm, cell, kPass == 0 ? kTagKeyE : kTagKeyG, rng, L.opn, L.opk, L.opj, n_open);
                if (t < n_open)
                    push_cand(W, c, ev_pack(kPass, (int)L.opj[t], (int)(L.opn[t] & 0xFFFFu), 0, L.opn[t] >> 16));
            }
        }
        }
        if (t == 0) W.coef[c * 2 + kPass] = coef;
    }
    if (t == 0) {
        if (kPass == 0) {
            A.ti[c * CMC_NI + CMC_I_PAIRS_BR] = (nab > 0.0 && (A.proc & CMC_BREMS)) ? N : 0;
            A.ti[c * CMC_NI + CMC_I_PAIRS_TR] = (nab > 0.0 && (A.proc & CMC_TRIDENT)) ? N : 0;
            A.td[c * CMC_ND + CMC_D_NAB_EI] = nab;
        } else {
            A.ti[c * CMC_NI + CMC_I_PAIRS_BH] = nab > 0.0 ? N : 0;
            A.td[c * CMC_ND + CMC_D_NAB_GI] = nab;
        }
    }
    if (team_any<kT>(high != 0, L.redi) && t == 0) atomicOr(A.status, CMC_ST_GAMMA_HIGH);
    Team<kT>::sync();   // LDS of this cell is free
}

// The pair tests of the cells whose ions are at rest and whose electrons
// each pair once (N_i <= N_e), above the direct form's size and up to the
// stream capacity `scap` (the LDS of one sigma v factor per electron, two
// with Trident): nothing depends on an order, and a cell is one walk over
// its records.  Every electron's momenta and weight and every ion's weight
// are read once, two records ahead of their use, while the walk forms each
// electron's FP32 test factor sigma v (into LDS) and the canonical
// per-thread parts of the densities and of n_ab (the order of canon_part2).
// The draws of U1's upper bits (one per four pairs) are made in the walk
// too, where the loads leave the ALUs idle, and each thread keeps the
// smallest kx at which one of its tests would pass the bound.  Once the
// team reduction gives kx, only a thread whose smallest value lies near or
// below it tests its pairs exactly as the pass kernel does, so the open
// pairs are the pass kernel's.
// kPh: the photon-ion pass of the same cell runs in the walk as well when
// its photons are cycled against the ions (0 < N_g < N_i, N_g <= 256): the
// photons' keys, ranks, repetitions, 1/(sigma c) and weight sums are formed
// before the walk, and its draws (one per four tests, 1024 for 4096 ions)
// are made inside it, filtered the same way.
// The open pairs are written to the cell's candidate records with their
// count (no atomics per pair); the cell is listed for the event kernels
// once, after the workgroup's last barrier.  Done passes are flagged
// (kFlagDone0, kFlagDone1); cells of unequal ion weights, and all others,
// are left to the pass kernel, marked in list_rest (a cell whose photon-ion
// pass is left, too).  One workgroup per cell, walking the cells in index
// order or (from_list 2) the work queue.
constexpr int kStreamPh = 256;   // photons per cell the stream kernel's photon-ion pass takes
constexpr int kLaneCap = 8;      // open pairs per cell the lane event kernel takes

// f(integral_constant<int, I>) for I = 0, 1, ... in order, unrolled
template <int... I, typename F>
__device__ __forceinline__ void unrolled(std::integer_sequence<int, I...>, F&& f) {
    (f(std::integral_constant<int, I>{}), ...);
}

// An electron record of the stream kernel's walk, and the ion weight beside it
struct Rec { double x, y, z, w, wi; };

// The two smallest values met, and the place of the smallest
struct Low {
    float y1 = INFINITY, y2 = INFINITY;
    int u1 = 0;
    __device__ __forceinline__ void add(float y, int u) {
        const bool lo = y < y1;
        y2 = lo ? y1 : fminf(y2, y);
        u1 = lo ? u : u1;
        y1 = lo ? y : y1;
    }
};

// A copy of v in registers of its own (an instruction the compiler cannot
// fold), so that the registers v arrived in may take the next load at once.
__device__ __forceinline__ double fresh(double v) {
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ Rec fresh(const Rec& r) {
    return Rec{fresh(r.x), fresh(r.y), fresh(r.z), fresh(r.w), fresh(r.wi)};
}

// 2^-24 2^24 w / s for the filter of the bound test (an upper bound on kx
// is not needed: the filter keeps a margin and the exact test decides)
__device__ __forceinline__ float kx_needed(uint32_t word, float s) {
    const uint32_t v = word >> 8;
    return v == 0u ? 0.0f : (float)v * __builtin_amdgcn_rcpf(s);
}

// The FP64 form's filter of the electron-ion bound test, in FP32: an upper
// bound of the Bremsstrahlung sigma that brems_sig_slice<double> gives for
// the same electron.  The energy axes of the three segments as FP32 values
// (start, reciprocal step, node count), selected by value per lane.
struct SegAxes {
    float u0[3], rdu[3];
    int n[3];
};

__host__ __device__ inline SegAxes seg_axes(const Axes& ax) {
    const AxisDef* a[3] = {&ax.nr, &ax.rel, &ax.ur};
    SegAxes S;
    for (int k = 0; k < 3; ++k) {
        S.u0[k] = (float)a[k]->u0;
        S.rdu[k] = (float)(1.0 / a[k]->du);
        S.n[k] = a[k]->n;
    }
    return S;
}

// The bound: the largest slice node of the interval the FP32 energy falls
// in and of its two neighbours.  The FP32 position along the axis differs
// from the FP64 one by far less than a node spacing (about 1e-4 of one), so
// the FP64 interval is among these three and its interpolated sigma is at
// most the largest of their nodes (which the FP32 copy of the slice holds
// rounded to nearest).  edge: the electron lies within 2^-10 (relative) of
// the emission threshold, of a segment join (gamma 2 and 100) or of the top
// of the tables, or its FP32 energy is not finite; there the two energies
// may fall on different sides, and the pair is tested exactly.  sl: the
// FP32 copy of the cell's slice (segments NR | rel | UR).
__device__ __forceinline__ float brems_sig_bound(const SegAxes& X, const float* sl, float g, float g1m1,
                                                 bool& edge) {
    constexpr float kB = 1.0f / 1024.0f;
    constexpr float tmin = (float)(grid::kTminEv / grid::kMec2Ev);
    edge = !(g < (float)grid::kTop * (1.0f - kB)) || fabsf(g - 2.0f) <= 2.0f * kB ||
           fabsf(g - 100.0f) <= 100.0f * kB || fabsf(g1m1 - tmin) <= tmin * kB;
    if (edge || !(g1m1 > tmin)) return 0.0f;
    const bool nr = g <= 2.0f, rel = g <= 100.0f;
    const float u0 = nr ? X.u0[0] : rel ? X.u0[1] : X.u0[2];
    const float rdu = nr ? X.rdu[0] : rel ? X.rdu[1] : X.rdu[2];
    const int n = nr ? X.n[0] : rel ? X.n[1] : X.n[2];
    const int off = nr ? 0 : rel ? grid::kNR : grid::kNR + grid::kRel;
    const float pos = (Fast<float>::log(nr ? g1m1 : g) - u0) * rdu;
    const int ig = pos <= 0.0f ? 0 : min((int)pos, n - 2);
    const float* s = sl + off;
    return fmaxf(fmaxf(s[max(ig - 1, 0)], s[ig]), fmaxf(s[ig + 1], s[min(ig + 2, n - 1)]));
}

template <typename R, bool kTri, bool kPh>
__global__ __launch_bounds__(kStreamThreads, kStreamWaves) void k_stream(StepArgs A, TabView<R> T, Work W, int scap,
                                                                       int from_list) {
    // Thread t stands for threads t + kST v, v < kV, of the 256-thread order
    // the canonical sums are defined in (canon_part2): its records u with
    // u mod kV = v are theirs, in the same order, and the partial sums of the
    // slot v are kept apart, so every sum is the one a workgroup of 256
    // threads forms.  Slot v of wavefront wv is the 256-thread order's
    // wavefront wv + kW v.
    constexpr int kST = kStreamThreads, kV = 256 / kST, kW = kST / 64;
    // FP64 form without Trident: the walk filters the bound tests with
    // brems_sig_bound in FP32, and a pair that passes the filter is tested
    // again from its FP64 sigma v, exactly as the pass kernel tests it
    constexpr bool kLoose = std::is_same<R, double>::value && !kTri;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ R slice[kSliceMax];
    __shared__ float slice_f[kLoose ? kSliceMax : 1];
    __shared__ R slice_g[kPh ? kSliceMax : 1];
    __shared__ double rs[4][4];                   // per wavefront of the 256 order: parts of n_e, n_ab, n_i
    __shared__ int rsf[kW];                       // per wavefront: flag bits
    __shared__ double pg[kPh ? 4 * 3 : 1];        // per wavefront of the 256 order: the photons' n_g, A, B parts
    __shared__ int pgf[kPh ? kW : 1];             // per wavefront: 1 bad photon weight, 4 above the tables
    __shared__ float pgm[kPh ? kW : 1];           // per wavefront: the smallest 1/(sigma c) of its photons
    __shared__ uint32_t opn[kCandCap];
    __shared__ int nopen;
    // the photons of the cell: key, then rank; repetitions; sigma and 1/(sigma c)
    __shared__ uint32_t gkey[kPh ? kStreamPh : 1];
    __shared__ uint16_t grank[kPh ? kStreamPh : 1], greps[kPh ? kStreamPh : 1];
    __shared__ float gsig[kPh ? kStreamPh : 1], ginv[kPh ? kStreamPh : 1];
    const int t = (int)threadIdx.x, lane = t & 63, wv = t >> 6;
    const double rej = 2.0 * (1.0 + A.near_rel);
    const Rng rng = step_rng(A);
    constexpr bool tri = kTri;
    const bool brm = (A.proc & CMC_BREMS) != 0;
    float* sv = reinterpret_cast<float*>(smem_raw);   // sigma v of electron q (< 0: no test)
    float* svt = sv + scap;                           // Trident's
    const SegAxes X3 = seg_axes(T.ax);
    for (int64_t item = blockIdx.x; item < A.n_cells; item += gridDim.x) {
        const int64_t c = from_list == 2 ? (int64_t)W.queue[item] : item;
        const uint32_t cell = cell_word(A.cid, c);
        const int32_t cstat = W.cs[c].status;
        const CellTab<R> ct = pick<R>(W.cs[c]);
        const int64_t e0 = A.el.off[c], eo1 = A.el.off[c + 1], g0 = A.ph.off[c], go1 = A.ph.off[c + 1];
        const int64_t i0 = A.io.off[c], io1 = A.io.off[c + 1];
        const int ecn = A.el.count ? A.el.count[c] : 0x7FFFFFFF, gcn = A.ph.count ? A.ph.count[c] : 0x7FFFFFFF;
        const int icn = A.io.count ? A.io.count[c] : 0x7FFFFFFF;
        const int Ne = max(0, min(ecn, (int)(eo1 - e0))), Ng = max(0, min(gcn, (int)(go1 - g0)));
        const int Ni = max(0, min(icn, (int)(io1 - i0)));
        // item's entry of list_rest: the cell, when a pass is left to the
        // pass kernel, else -1 (the pass kernel walks the entries in the
        // order of this walk: index order, or the work queue's)
        const auto rest = [&](bool left) {
            if (t == 0) {
                W.list_rest[item] = left ? (int32_t)c : -1;
                if (left) atomicAdd(&W.counters[kCntRest], 1);
            }
        };
        if (cstat) {                             // invalid cell (flagged by k_cell_state)
            rest(false);
            continue;
        }
        if (Ni == 0 || Ne < Ni || Ne <= 1024 || Ne > scap || Ne > A.maxn || Ng > A.maxn) {
            rest(true);
            continue;
        }
        const int N = Ne, U = (N + kST - 1) / kST;
        const double* wm = A.el.w + e0;
        const double* wion = A.io.w + i0;
        const double* wo = A.ph.w + g0;
        const auto load = [&](int u) {
            const int q = min(t + kST * u, N - 1), qi = min(t + kST * u, Ni - 1);
            return Rec{A.el.px[e0 + q], A.el.py[e0 + q], A.el.pz[e0 + q], wm[q], wion[qi]};
        };
        // the photon-ion pass here: photons cycled against the ions (the pair
        // count is N_i; photon m pairs K = N_i div N_g times and, if its rank
        // is below e = N_i mod N_g, once more, keys x = m + k N_g < X)
        const bool ph = kPh && Ng > 0 && Ng < Ni && Ng <= kStreamPh;
        const bool left1 = !ph && (A.proc & CMC_BH) && Ng > 0;      // a photon-ion pass for the pass kernel
        const int K = ph ? Ni / Ng : 0, ee = ph ? Ni - K * Ng : 0;
        const int X = K * Ng + (ee > 0 ? Ng : 0);
        const int Gt = ph ? (((X + 1023) >> 10) << 8) / kST : 0;   // draw groups per thread
        const float rNg = ph ? 1.0f / (float)Ng : 0.0f;
        // Loads in the order their values are needed: the table slices (from
        // L2) first, then the photons, then the first electron records,
        // which stay in flight through the staging and the photons' setup.
        if (brm)
            for (int i = t; i < kSliceBrems; i += kST) {
                const R sn = slice_node_brems<R>(T, ct, i);
                slice[i] = sn;
                if constexpr (kLoose) slice_f[i] = (float)sn;
            }
        if (ph)
            for (int i = t; i < kSliceBH; i += kST) slice_g[i] = slice_node_bh<R>(T, ct, i);
        double gw[kV], gx[kV], gy[kV], gz[kV];                  // this thread's photons m = t + kST v
#pragma unroll
        for (int v = 0; v < kV; ++v) {
            const int m = t + kST * v;
            gw[v] = 0.0; gx[v] = 0.0; gy[v] = 0.0; gz[v] = 0.0;
            if (ph && m < Ng) {
                gx[v] = A.ph.px[g0 + m]; gy[v] = A.ph.py[g0 + m]; gz[v] = A.ph.pz[g0 + m];
                gw[v] = wo[m];
            }
        }
        const double w0 = wion[0];
        Rec rr[kStreamDepth];
#pragma unroll
        for (int d = 0; d < kStreamDepth; ++d) rr[d] = load(min(d, U - 1));
        if (ph)
            for (int m = t; m < Ng; m += kST) gkey[m] = hi_word(rng.draw((uint32_t)m >> 2, cell, kTagKeyG), (uint32_t)m & 3u);
        if (t == 0) nopen = 0;
        __syncthreads();
        if (ph) {
            // rank of photon t by (key, index); its tests; sigma and 1/(sigma c);
            // the canonical per-wavefront parts of n_g, A = sum min(W_g, W_i)
            // and B, the same over the photons that pair once more
            int flg = 0;
            float imin = INFINITY;
#pragma unroll
            for (int v = 0; v < kV; ++v) {
                const int mt = t + kST * v;
                double pa = 0.0, pb = 0.0, pc = 0.0;
                if (mt < Ng) {
                    const uint32_t kt = gkey[mt];
                    int rk = 0;
                    for (int j = 0; j < Ng; ++j) {
                        const uint32_t kj = gkey[j];
                        rk += (kj < kt || (kj == kt && j < mt)) ? 1 : 0;
                    }
                    grank[mt] = (uint16_t)rk;
                    greps[mt] = (uint16_t)(K + (rk < ee ? 1 : 0));
                    bool hi;
                    const R sig = bh_sig_slice<R>(T, slice_g, photon_k<R>(gx[v], gy[v], gz[v]), hi);
                    flg |= hi ? 4 : 0;
                    gsig[mt] = (float)sig;
                    ginv[mt] = sig > (R)0 ? 1.0f / ((float)sig * (float)phys::kC) : -1.0f;
                    if (sig > (R)0) imin = fminf(imin, ginv[mt]);
                    flg |= (!(gw[v] >= 0.0) || !isfinite(gw[v])) ? 1 : 0;
                    const double m = gw[v] < w0 ? gw[v] : w0;
                    pa = 0.0 + gw[v];
                    pb = 0.0 + m;
                    pc = rk < ee ? 0.0 + m : 0.0;
                }
                pa = wave_sum(pa);
                pb = wave_sum(pb);
                pc = wave_sum(pc);
                if (lane == 0) {
                    pg[(wv + kW * v) * 3] = pa;
                    pg[(wv + kW * v) * 3 + 1] = pb;
                    pg[(wv + kW * v) * 3 + 2] = pc;
                }
            }
            const int f1 = __ballot(flg & 1) != 0ull ? 1 : 0, f4 = __ballot(flg & 4) != 0ull ? 4 : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) imin = fminf(imin, __shfl_xor(imin, o, 64));
            if (lane == 0) { pgf[wv] = f1 | f4; pgm[wv] = imin; }
            __syncthreads();
        }
        // the filter of the photon-ion tests bounds every test with the
        // largest sigma of the cell's photons: v / (sigma_max c) is at most
        // the test's own v / (sigma c), so no test that passes is missed
        // (the exact tests follow for a thread whose bound passes)
        float ginv_min = INFINITY;
        if (ph)
#pragma unroll
            for (int w = 0; w < kW; ++w) ginv_min = fminf(ginv_min, pgm[w]);
        double sa[kV], sb[kV], si[kV];           // n_e, n_ab and n_i: canonical parts of the slots
#pragma unroll
        for (int v = 0; v < kV; ++v) { sa[v] = 0.0; sb[v] = 0.0; si[v] = 0.0; }
        int fl = 0;                              // 1 bad weight, 2 ions of unequal weight, 4 above the tables
        // the two smallest kx at which one of this thread's tests would pass
        // the bound, with the word and place of the smallest: Bremsstrahlung,
        // Trident, Bethe-Heitler
        Low lb, lt, lg;
        U4 hb[kV], ht[kV];
        // draw group j of this thread's photon-ion tests: g = t + kST j, keys base(g) + 256 w
        const auto group = [&](int j) {
            const int g = t + kST * j;
            const int base = ((g >> 8) << 10) | (g & 255);
            if (base >= X) return;
            const U4 h = rng.draw((uint32_t)g, cell, kTagHiBh);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int x = base + 256 * w;
                if (x >= X) break;
                const uint32_t v = hi_word(h, (uint32_t)w) >> 8;
                lg.add(v == 0u ? 0.0f : (float)v * ginv_min, x);
            }
        };
        // record u of the walk (q = t + kST u), slot v = u mod kV
        const auto take = [&](int u, const Rec& cur, auto vc) {
            constexpr int v = decltype(vc)::value;
            const int q = t + kST * u, vu = u / kV;
            // pair q: U1's upper bits are word vu & 3 of the draw
            // hi_group(q) = (vu >> 2) << 8 | (t + kST v), one per four pairs
            if ((vu & 3) == 0) {
                if (brm) hb[v] = rng.draw(hi_group((uint32_t)q), cell, kTagHiBr);
                if (tri) ht[v] = rng.draw(hi_group((uint32_t)q), cell, kTagHiTr);
            }
            if (q < N) {
                fl |= (!(cur.w >= 0.0) || !isfinite(cur.w)) ? 1 : 0;
                sa[v] += cur.w;
                sb[v] += cur.w < w0 ? cur.w : w0;
                if constexpr (kLoose) {
                    if (brm) {
                        // an edge electron passes the filter (it is tested exactly)
                        const Elec<float> ef = electron_p<float>(cur.x, cur.y, cur.z);
                        bool edge;
                        const float sup = brems_sig_bound(X3, slice_f, ef.g, ef.gm1, edge);
                        if (edge || sup > 0.0f)
                            lb.add(edge ? 0.0f : kx_needed(hi_word(hb[v], (uint32_t)vu & 3u), sup * (float)ef.vrel), u);
                    }
                } else {
                    const Elec<R> el = electron_p<R>(cur.x, cur.y, cur.z);
                    float s1 = -1.0f;
                    if (brm) {
                        bool hi;
                        const R sig = brems_sig_slice<R>(T, slice, el.g, el.gm1, hi);
                        fl |= hi ? 4 : 0;
                        if (sig > (R)0) {
                            s1 = (float)sig * (float)el.vrel;
                            lb.add(kx_needed(hi_word(hb[v], (uint32_t)vu & 3u), s1), u);
                        }
                    }
                    sv[q] = s1;
                    if (tri) {
                        const R st = (R)phys::trident_sigma(T.Z, (double)el.g);
                        float s2 = -1.0f;
                        if (st > (R)0) {
                            s2 = (float)st * (float)el.vrel;
                            lt.add(kx_needed(hi_word(ht[v], (uint32_t)vu & 3u), s2), u);
                        }
                        svt[q] = s2;
                    }
                }
            }
            if (q < Ni) {
                fl |= (!(cur.wi >= 0.0) || !isfinite(cur.wi)) ? 1 : 0;
                fl |= cur.wi != w0 ? 2 : 0;
                si[v] += cur.wi;
            }
            if (ph && (u & 3) == 3 && (u >> 2) < Gt) group(u >> 2);
        };
        // kStreamDepth records in flight per thread, each in registers of its
        // own: the walk takes kStreamDepth records a round, each copied out
        // (fresh, once it has arrived) before the load of the record
        // kStreamDepth ahead goes out into its registers.  A plain rotation
        // (r0 = r1) would move a value still in flight, which waits for every
        // load.  The last round's loads are clamped to the last record.
        static_assert(kStreamDepth % kV == 0, "a round of records covers whole slots");
#pragma unroll 1
        for (int u0 = 0; u0 < U; u0 += kStreamDepth) {
            unrolled(std::make_integer_sequence<int, kStreamDepth>{}, [&](auto dc) {
                constexpr int d = decltype(dc)::value;
                const Rec cur = fresh(rr[d]);
                rr[d] = load(min(u0 + d + kStreamDepth, U - 1));
                if (u0 + d < U) take(u0 + d, cur, std::integral_constant<int, d % kV>{});
            });
        }
        if (ph)
            for (int j = U >> 2; j < Gt; ++j) group(j);
        {
            // the team reduction: per-wavefront parts, one barrier (which also
            // publishes sv), the four parts added in order
            if (!ph)   // the photons' weights are checked (their pass is left to the pass kernel)
                for (int q = t; q < Ng; q += kST) fl |= (!(wo[q] >= 0.0) || !isfinite(wo[q])) ? 1 : 0;
#pragma unroll
            for (int v = 0; v < kV; ++v) {
                const double p0 = wave_sum(sa[v]), p1 = wave_sum(sb[v]), p2 = wave_sum(si[v]);
                if (lane == 0) {
                    rs[wv + kW * v][0] = p0;
                    rs[wv + kW * v][1] = p1;
                    rs[wv + kW * v][2] = p2;
                }
            }
            int wf = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (__ballot((fl >> b) & 1) != 0ull) wf |= 1 << b;
            if (lane == 0) rsf[wv] = wf;
            __syncthreads();
        }
        double v4[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) v4[k] = ((rs[0][k] + rs[1][k]) + rs[2][k]) + rs[3][k];
        fl = 0;
#pragma unroll
        for (int w = 0; w < kW; ++w) fl |= rsf[w];
        int flg = 0;
        if (ph) {
#pragma unroll
            for (int w = 0; w < kW; ++w) flg |= pgf[w];
            fl |= flg & 1;
        }
        if (fl & 2) {                                // the ordered form, in the pass kernel
            rest(true);
            __syncthreads();                         // rs is read by every thread
            continue;
        }
        if (fl & 1) {
            // bad weights: flagged, and the pass kernel skips the cell's passes done here
            if (t == 0) {
                atomicOr(A.status, CMC_ST_BAD_WEIGHT);
                atomicOr(&W.flags[c], kFlagDone0 | (ph ? kFlagDone1 : 0));
            }
            rest(left1);
            __syncthreads();
            continue;
        }
        int nc = 0;                                  // candidate records written
        const double nab = v4[1];
        if (nab > 0.0) {
            const double coef = v4[0] * v4[2] / nab;
            const float kx = (float)(coef * A.dt * rej * 16777216.0);
            const float kxf = kx * 1.001f;           // the filter's margin over the roundings of kx_needed
            // the exact test of the pass kernel: every pair of the thread when
            // two of them pass the filter, else the one that does
            const auto open_pair = [&](int q, uint32_t bits) {
                const int o = atomicAdd(&nopen, 1);
                if (o < kCandCap) opn[o] = (uint32_t)q | (bits << 16);
            };
            // electron q's Bremsstrahlung sigma v as the pass kernel forms it
            // (< 0: no test): from LDS, or (kLoose) from its FP64 momenta,
            // which also decide whether it lies above the tables
            const auto sig_v = [&](int q) -> float {
                if constexpr (kLoose) {
                    const int64_t ie = e0 + q;
                    const Elec<R> el = electron_p<R>(A.el.px[ie], A.el.py[ie], A.el.pz[ie]);
                    bool hi;
                    const R sig = brems_sig_slice<R>(T, slice, el.g, el.gm1, hi);
                    if (hi) atomicOr(A.status, CMC_ST_GAMMA_HIGH);
                    return sig > (R)0 ? (float)sig * (float)el.vrel : -1.0f;
                } else {
                    return sv[q];
                }
            };
            if (lb.y2 <= kxf || lt.y2 <= kxf) {
                // each pair's word drawn on its own (this path is rare)
                for (int u = 0; u < U; ++u) {
                    const int q = t + kST * u;
                    if (q >= N) continue;
                    uint32_t bits = 0;
                    const float s1 = brm ? sig_v(q) : -1.0f;
                    if (s1 > 0.0f &&
                        bound24(hi_word(rng.draw(hi_group((uint32_t)q), cell, kTagHiBr), ((uint32_t)q >> 8) & 3u), kx * s1))
                        bits = 1u;
                    if (tri && !bits) {
                        const float s2 = svt[q];
                        if (s2 > 0.0f &&
                            bound24(hi_word(rng.draw(hi_group((uint32_t)q), cell, kTagHiTr), ((uint32_t)q >> 8) & 3u), kx * s2))
                            bits = 2u;
                    }
                    if (bits) open_pair(q, bits);
                }
            } else {
                // Bremsstrahlung first, Trident where it fails; every other pair
                // of the thread fails both filters, hence both tests.  The
                // pair's word is drawn again.
                const auto word = [&](int u, uint32_t tag) {
                    const uint32_t q = (uint32_t)(t + kST * u);
                    return hi_word(rng.draw(hi_group(q), cell, tag), (q >> 8) & 3u);
                };
                bool done_t = false;
                if (lb.y1 <= kxf) {
                    const int q = t + kST * lb.u1;
                    const float s1 = sig_v(q);
                    if (s1 > 0.0f && bound24(word(lb.u1, kTagHiBr), kx * s1)) {
                        open_pair(q, 1u);
                        done_t = tri && lt.u1 == lb.u1;
                    }
                }
                if (tri && !done_t && lt.y1 <= kxf) {
                    const int q = t + kST * lt.u1;
                    if (bound24(word(lt.u1, kTagHiTr), kx * svt[q])) open_pair(q, 2u);
                }
            }
            __syncthreads();
            nc = nopen;
            if (nc > 0 && nc <= kCandCap && t < 64) {
                // The event kernels use an open pair's index only to order the
                // open pairs of a pass: every electron here pairs once, with
                // interchangeable ions, so a pair's draws are keyed by its
                // electron alone and nothing else depends on the index.  Its
                // rank among the open pairs by (key, electron) orders them as
                // the pair indices do, and stands for the index.
                const bool has = t < nc;
                const uint32_t mt = has ? (opn[t] & 0xFFFFu) : 0u;
                uint32_t kt = 0u;
                if (has) kt = hi_word(rng.draw(mt >> 2, cell, kTagKeyE), mt & 3u);
                int rk = 0;
                for (int j = 0; j < nc; ++j) {
                    const uint32_t kj = (uint32_t)__builtin_amdgcn_readlane((int)kt, j);
                    const uint32_t mj = (uint32_t)__builtin_amdgcn_readlane((int)mt, j);
                    rk += (kj < kt || (kj == kt && mj < mt)) ? 1 : 0;
                }
                if (has) W.cand[c * kCandCap + t] = ev_pack(0, rk, (int)mt, 0, opn[t] >> 16);
            }
            if (t == 0) W.coef[c * 2] = coef;
        }
        if (ph) {
            const double ng = ((pg[0] + pg[3]) + pg[6]) + pg[9];
            const double Ag = ((pg[1] + pg[4]) + pg[7]) + pg[10];
            const double Bg = ((pg[2] + pg[5]) + pg[8]) + pg[11];
            const double nabg = fma((double)K, Ag, Bg);   // as the pass kernel forms it
            if (nabg > 0.0) {
                const double coefg = ng * v4[2] / nabg;
                const float kxg = (float)(coefg * A.dt * rej * 16777216.0);
                const float kxgf = kxg * 1.001f;
                const bool any = __syncthreads_or(lg.y1 <= kxgf) != 0;
                if (any) {
                    // the photon-ion tests again with the pass kernel's bound
                    if (t == 0) nopen = 0;
                    __syncthreads();
                    const auto test = [&](int x, uint32_t wd) {
                        const int m = mod_small(x, Ng, rNg);
                        const int k = __float2int_rn((float)(x - m) * rNg);
                        const float sg = gsig[m];
                        if (k < (int)greps[m] && sg > 0.0f && bound24(wd, kxg * sg * (float)phys::kC)) {
                            const int o = atomicAdd(&nopen, 1);
                            if (o < kCandCap) opn[o] = (uint32_t)m | ((uint32_t)k << 16);
                        }
                    };
                    if (lg.y2 <= kxgf) {
                        for (int j = 0; j < Gt; ++j) {
                            const int g = t + kST * j;
                            const int base = ((g >> 8) << 10) | (g & 255);
                            if (base >= X) continue;
                            const U4 h = rng.draw((uint32_t)g, cell, kTagHiBh);
                            for (int w = 0; w < 4; ++w) {
                                const int x = base + 256 * w;
                                if (x >= X) break;
                                test(x, hi_word(h, (uint32_t)w));
                            }
                        }
                    } else if (lg.y1 <= kxgf) {
                        // the key's word, drawn again
                        const int x = lg.u1;
                        const int g = ((x >> 10) << 8) | (x & 255);
                        test(x, hi_word(rng.draw((uint32_t)g, cell, kTagHiBh), (uint32_t)(x >> 8) & 3u));
                    }
                    __syncthreads();
                    const int ngo = nopen;
                    if (ngo > 0 && nc + ngo <= kCandCap && t < ngo) {
                        // pair index: the photon's rank plus k N_g
                        const uint32_t o = opn[t];
                        const int m = (int)(o & 0xFFFFu), k = (int)(o >> 16);
                        W.cand[c * kCandCap + nc + t] = ev_pack(1, (int)grank[m] + k * Ng, m, 0, 1u);
                    }
                    nc += ngo;
                }
                if (t == 0) W.coef[c * 2 + 1] = coefg;
            }
            if (t == 0) {
                A.ti[c * CMC_NI + CMC_I_PAIRS_BH] = nabg > 0.0 ? Ni : 0;
                A.td[c * CMC_ND + CMC_D_NAB_GI] = nabg;
                if (nabg > 0.0 && (flg & 4)) atomicOr(A.status, CMC_ST_GAMMA_HIGH);
            }
        }
        if (t == 0) {
            A.ti[c * CMC_NI + CMC_I_PAIRS_BR] = (nab > 0.0 && brm) ? N : 0;
            A.ti[c * CMC_NI + CMC_I_PAIRS_TR] = (nab > 0.0 && tri) ? N : 0;
            A.td[c * CMC_ND + CMC_D_NAB_EI] = nab;
            if (nab > 0.0 && (fl & 4)) atomicOr(A.status, CMC_ST_GAMMA_HIGH);
            W.ionsum[c] = v4[2];
            W.ncand[c] = nc;
        }
        __syncthreads();   // LDS of this cell is free
        if (t == 0) {
            // flags, then the lists (the only waits on atomics, after the barrier)
            // a cell whose open pairs are a few electron-ion pairs, with no
            // photon-ion pass left and no Trident, goes to the lane kernel
            const int32_t f = kFlagWeightsOk | kFlagIonsSame | kFlagDone0 | (ph ? kFlagDone1 : 0) |
                              (nc > kCandCap ? kFlagSlow : 0) | (nc > 0 ? kFlagListed : 0);
            if (nc > 0) {
                const bool by_lane = nc <= kLaneCap && !tri && !left1;
                if (!(atomicOr(&W.flags[c], f) & kFlagListed)) {
                    if (by_lane) W.list_lane[atomicAdd(&W.counters[kCntLane], 1)] = (int32_t)c;
                    else W.list_ev[atomicAdd(&W.counters[kCntEv], 1)] = (int32_t)c;
                }
            } else {
                atomicOr(&W.flags[c], f);
            }
        }
        rest(left1);
    }
}

// One pass of pair tests over all cells from the particles as they are at
// One pass of pair tests over all cells from the particles as they are at
// the start of the step: kPass 0 electron-ion (Bremsstrahlung, then Trident
// when Bremsstrahlung is not accepted), kPass 1 photon-ion (Bethe-Heitler),
// kPass 2 both, one after the other by the same team for each cell (the
// photon-ion pass then takes the ions' weight sum from the electron-ion
// pass in registers, and its latency-bound work overlaps the streaming of
// the other teams on the compute unit).
// A test is settled here when U1 > 2 (1 + near_rel) x: then P <= x < U1 and
// |U1 - P| > near_rel P hold for the computed values, so the pair has no
// event and no near-threshold count whatever P is.  The rare other pairs are
// listed and settled with P by the event kernel.
// kMov: the ions move, and each pair is tested in its ion's rest frame.
// Workgroup teams run best at six wavefronts per SIMD (a few spilled
// registers); wavefront teams are limited by LDS anyway.
// LDS: `cap` particles per species fit the team's sort arrays.  A pass
// whose cell exceeds that but needs no order (ions at rest sharing one
// weight, every mobile particle paired once) runs here all the same; one
// that needs an order larger than cap is deferred to list_big[kPass],
// which a launch with a larger cap walks (from_list = 1).  Cells above
// slow_cap, the largest cap of the step, take the sequential step whole.
template <typename R, int kT, int kPass, bool kMov, bool kRest = false>
__global__ __launch_bounds__(256, kT == 256 ? 6 : 1) void k_pass(StepArgs A, TabView<R> T, Work W, int cap, int filter, int fcap,
                                                                 int slow_cap, int from_list) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red4[kWaves * 4];
    __shared__ uint32_t redu[kWaves];
    __shared__ int redi[kWaves];
    constexpr int kTeams = 256 / kT;
    __shared__ uint32_t opn[kTeams][kCandCap];    // open pairs found without the order
    __shared__ uint32_t opk[kTeams][kCandCap];    // their particles' keys
    __shared__ uint32_t opj[kTeams][kCandCap];    // their pair indices
    __shared__ int nopen[kTeams];
    __shared__ int32_t rest_ent[kRest ? 256 : 1];             // per thread: its list_rest entry of the batch
    __shared__ unsigned long long rest_mask[kRest ? 4 : 1];   // per wavefront: the entries >= 0
    const int team = kT == 64 ? (int)(threadIdx.x >> 6) : 0;
    const int t = Team<kT>::tid();
    const size_t tstride = (team_bytes(cap, (int)sizeof(R), kT) + 15) / 16 * 16;
    const TeamMem M = carve_team(smem_raw + tstride * team, cap, kT);
    const double rej = 2.0 * (1.0 + A.near_rel);
    const Rng rng = step_rng(A);

    const PassLds L{red4, redu, redi, opn[team], opk[team], opj[team], &nopen[team]};
    // from_list 0: every cell in index order; 1: the pass's deferred list;
    // 3: the cells the stream kernel left, in the order of its walk;
    // 2: the work queue, the cells costliest first (workgroups are
    // dispatched in index order as compute units free up, so the largest
    // cells start first and the rest fill in behind them)
    // The walk of list_rest ends at once when the stream kernel left no
    // cell.  (Folded into the choice of n_items below, as a nested
    // conditional, this test made the compiler drop n_cells on the path where
    // the count is not zero: the early return keeps the two apart.)
    if ((kRest || from_list == 3) &&
        __hip_atomic_load(&W.counters[kCntRest], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;
    if constexpr (kRest) {
        // from_list 3 (its own instantiation, so that the other lists keep
        // their plain loop): the team's items are item0 + k G (G teams in
        // the grid, which holds only the teams that fit on the device at
        // once); their list_rest entries are read kT at a time, one per
        // thread, and the cells among them (entries >= 0: the cells the
        // stream kernel left) run in item order
        const int64_t G = (int64_t)gridDim.x * kTeams;
        for (int64_t i0 = (int64_t)blockIdx.x * kTeams + team; i0 < A.n_cells; i0 += G * kT) {
            const int64_t it = i0 + (int64_t)t * G;
            const int32_t e = it < A.n_cells ? W.list_rest[it] : -1;
            const unsigned long long mk = __ballot(e >= 0);
            rest_ent[threadIdx.x] = e;
            if ((t & 63) == 0) rest_mask[threadIdx.x >> 6] = mk;
            Team<kT>::sync();
            for (int w = 0; w < kT / 64; ++w) {
                // the mask and the cell as wave-uniform values (scalar registers)
                const int wave = kT == 64 ? team : w;
                const unsigned long long mw = rest_mask[wave];
                unsigned long long m =
                    ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(mw >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)mw);
                for (; m; m &= m - 1ull) {
                    const int64_t c = __builtin_amdgcn_readfirstlane(rest_ent[wave * 64 + __ffsll((long long)m) - 1]);
                    PassCarry carry{0, 0.0};
                    if constexpr (kPass != 1)
                        pass_cell<R, kT, 0, kMov, false>(A, T, W, cap, filter, fcap, slow_cap, c, M, rng, rej, t, L,
                                                         carry);
                    if constexpr (kPass != 0)
                        pass_cell<R, kT, 1, kMov, kPass == 2>(A, T, W, cap, filter, fcap, slow_cap, c, M, rng, rej, t,
                                                              L, carry);
                }
            }
            Team<kT>::sync();   // the entries are read before the next batch
        }
    } else {
        const int64_t n_items = from_list == 1 ? (int64_t)W.counters[kPass == 1 ? kCntBig1 : kCntBig0] : A.n_cells;
        for (int64_t item = (int64_t)blockIdx.x * kTeams + team; item < n_items; item += (int64_t)gridDim.x * kTeams) {
            const int64_t c = from_list == 2 ? (int64_t)W.queue[item]
                            : from_list == 3 ? (int64_t)W.list_rest[item]
                            : from_list ? (int64_t)W.list_big[kPass == 1 ? 1 : 0][item] : item;
            if (c < 0) continue;                     // done by the stream kernel
            PassCarry carry{0, 0.0};
            if constexpr (kPass != 1)
                pass_cell<R, kT, 0, kMov, false>(A, T, W, cap, filter, fcap, slow_cap, c, M, rng, rej, t, L, carry);
            if constexpr (kPass != 0)
                pass_cell<R, kT, 1, kMov, kPass == 2>(A, T, W, cap, filter, fcap, slow_cap, c, M, rng, rej, t, L, carry);
        }
    }
}

// The work queue of the batched schedule: the cells in decreasing order
// of their cost in the pass kernel, the pairs of both passes (max(N_a, N_b)
// each) plus a fixed per-cell term, counted into buckets of a quarter
// octave, costliest first.  The order within a bucket is whatever the
// atomics give: no result depends on which team runs which cell when.
// One workgroup: the counts are read twice rather than stored.
constexpr int kQBuckets = 128;
constexpr int kQThreads = 1024;

// Cost bucket of a cell with Ne, Ng, Ni live particles: a quarter octave
// of 64 + the pairs of its two passes
__device__ __forceinline__ int queue_bucket(const StepArgs& A, int Ne, int Ng, int Ni) {
    const bool ei = (A.proc & (CMC_BREMS | CMC_TRIDENT)) && Ne > 0 && Ni > 0;
    const bool gi = (A.proc & CMC_BH) && Ng > 0 && Ni > 0;
    const uint32_t cost = 64u + (ei ? (uint32_t)max(Ne, Ni) : 0u) + (gi ? (uint32_t)max(Ng, Ni) : 0u);
    const int b = 31 - __clz((int)cost);                     // cost >= 64: b >= 6
    return min(kQBuckets - 1, 4 * b + (int)((cost >> (b - 2)) & 3u));
}

// The live counts of one species in kQCells cells (c[u], all valid), every
// load issued before the first is used.  Without live counts the words
// read in their place are the offsets' own (in bounds: the offsets hold
// 2 (n_cells + 1) words) and are not used, so that no branch separates
// the loads.
constexpr int kQCells = 4;
__device__ __forceinline__ void queue_live(const SpeciesDev& S, const int64_t (&c)[kQCells], int (&n)[kQCells]) {
    const bool has = S.count != nullptr;
    const int32_t* cnt = has ? S.count : reinterpret_cast<const int32_t*>(S.off);
    int64_t lo[kQCells], hi[kQCells];
#pragma unroll
    for (int u = 0; u < kQCells; ++u) { lo[u] = S.off[c[u]]; hi[u] = S.off[c[u] + 1]; n[u] = cnt[c[u]]; }
#pragma unroll
    for (int u = 0; u < kQCells; ++u) {
        const int cap = (int)(hi[u] - lo[u]);
        n[u] = !has ? cap : n[u] < 0 ? 0 : (n[u] > cap ? cap : n[u]);
    }
}

// The buckets of the kQCells cells c0, c0 + kQThreads, ... of a thread (-1
// past the end), their loads issued together (read one cell at a time,
// each load waited for before the next, the launch was a chain of memory
// latencies).  Positions past the end read the last cell.
__device__ __forceinline__ void queue_buckets(const StepArgs& A, int64_t c0, int (&b)[kQCells]) {
    int64_t c[kQCells];
#pragma unroll
    for (int u = 0; u < kQCells; ++u) {
        const int64_t cu = c0 + (int64_t)u * kQThreads;
        c[u] = cu < A.n_cells ? cu : A.n_cells - 1;
    }
    int ne[kQCells], ng[kQCells], ni[kQCells];
    queue_live(A.el, c, ne);
    queue_live(A.ph, c, ng);
    queue_live(A.io, c, ni);
#pragma unroll
    for (int u = 0; u < kQCells; ++u)
        b[u] = c0 + (int64_t)u * kQThreads < A.n_cells ? queue_bucket(A, ne[u], ng[u], ni[u]) : -1;
}

__global__ __launch_bounds__(kQThreads) void k_queue(StepArgs A, Work W) {
    __shared__ int hist[kQBuckets];
    __shared__ int base[kQBuckets];
    const int t = threadIdx.x;
    constexpr int64_t kStride = (int64_t)kQThreads * kQCells;
    for (int b = t; b < kQBuckets; b += kQThreads) hist[b] = 0;
    __syncthreads();
    for (int64_t c0 = t; c0 < A.n_cells; c0 += kStride) {
        int b[kQCells];
        queue_buckets(A, c0, b);
#pragma unroll
        for (int u = 0; u < kQCells; ++u)
            if (b[u] >= 0) atomicAdd(&hist[b[u]], 1);
    }
    __syncthreads();
    if (t < kQBuckets) {
        int s = 0;
        for (int b = kQBuckets - 1; b > t; --b) s += hist[b];
        base[t] = s;
    }
    __syncthreads();
    for (int64_t c0 = t; c0 < A.n_cells; c0 += kStride) {
        int b[kQCells];
        queue_buckets(A, c0, b);
#pragma unroll
        for (int u = 0; u < kQCells; ++u)
            if (b[u] >= 0) W.queue[atomicAdd(&base[b[u]], 1)] = (int32_t)(c0 + (int64_t)u * kQThreads);
    }
}

// The values an event kernel reads for a listed cell, in one round of
// loads (each later round of dependent reads costs the chain about a
// microsecond), and this lane's open-pair record.
template <typename R>
struct EvCell {
    int64_t c, g0, e0, i0, ne0, np0;
    int Ng0, Ne, Ni, cap_ph, cap_ne, cap_np, cnt_ne0, cnt_np0, ncr, nc;
    int32_t flg;
    CellTab<double> ct64;
    CellTab<R> ct;
    double coef0, coef1;
    uint32_t cell;
    uint64_t raw;
};

template <typename R>
__device__ __forceinline__ EvCell<R> ev_cell(const StepArgs& A, const Work& W, int64_t c, int lane) {
    EvCell<R> E;
    E.c = c;
    E.flg = W.flags[c];
    E.ncr = W.ncand[c];
    E.raw = W.cand[c * kCandCap + lane];
    E.g0 = A.ph.off[c]; E.e0 = A.el.off[c]; E.i0 = A.io.off[c];
    E.Ng0 = live(A.ph, c); E.Ne = live(A.el, c); E.Ni = live(A.io, c);
    E.cap_ph = (int)(A.ph.off[c + 1] - E.g0);
    E.ne0 = A.ne.off[c]; E.np0 = A.np.off[c];
    E.cap_ne = (int)(A.ne.off[c + 1] - E.ne0);
    E.cap_np = (int)(A.np.off[c + 1] - E.np0);
    E.cnt_ne0 = A.ne.count[c]; E.cnt_np0 = A.np.count[c];
    E.ct64 = W.cs[c].d;
    E.ct = pick<R>(W.cs[c]);
    E.coef0 = W.coef[c * 2]; E.coef1 = W.coef[c * 2 + 1];
    E.cell = cell_word(A.cid, c);
    E.nc = min(E.ncr, kCandCap);
    return E;
}

// One open pair per lane of a wavefront, in (pass, pair index) order, once
// settled: its pair and particles, the event kind, and what the sampling
// of its event needs (the mobile particle seen from the ion, the FP64
// lookup).
template <typename R>
struct EvLane {
    int pass, j, mi, ii;
    uint32_t dk, kind;
    int near_br, near_tr, near_bh;
    double px, py, pz, Wm, Wi;
    Ion b;
    Frame fr;
    BremsLook<double> BLd;
    int ikd;
    double wkd;
    bool reused;
    bool last;     // no later event of its pass on the same particle
};

// Settles one open pair (record `mine`, or none when !cand) with P: the
// same arithmetic as the pass kernels (lookups from the full tables give
// the same values as the slices).  `reused` marks an open pair whose mobile
// particle is used by a later pair of its pass.
template <typename R>
__device__ __forceinline__ EvLane<R> ev_pair(const StepArgs& A, const TabView<R>& T, const TabView<double>& T64,
                                             const Rng& rng, const EvCell<R>& E, uint64_t mine, bool cand,
                                             double rej) {
    EvLane<R> L{};
    L.pass = cand ? ev_pass(mine) : 2;
    L.b = Ion{0.0, 0.0, 0.0, 1.0, false};
    L.j = ev_j(mine); L.mi = ev_m(mine); L.ii = ev_i(mine);
    // the pair's draws: keyed by its mobile particle and its repetition
    {
        const int nm = L.pass == 0 ? E.Ne : E.Ng0;
        L.dk = cand && nm > 0 ? (uint32_t)(L.mi + (L.j / nm) * nm) : 0u;
    }
    L.reused = false;
    L.last = true;
    if (cand) {
        const uint32_t bits = ev_kind(mine);
        const double coef = L.pass == 0 ? E.coef0 : E.coef1;
        L.Wi = A.io.w[E.i0 + L.ii];
        L.b = ion_at(A.io, E.i0 + L.ii);
        if (L.pass == 0) {
            const int64_t ie = E.e0 + L.mi;
            L.px = A.el.px[ie]; L.py = A.el.py[ie]; L.pz = A.el.pz[ie]; L.Wm = A.el.w[ie];
            L.fr = electron_frame(L.b, L.px, L.py, L.pz);
            const Elec<R> e = L.b.mov ? electron_moving<R>(L.fr, L.b) : electron_p<R>(L.px, L.py, L.pz);
            const double Pej = L.Wi / (L.Wm > L.Wi ? L.Wm : L.Wi);
            if (bits & 1u) {
                bool hi2;
                L.BLd = brems_lookup<double, false>(T64, E.ct64, L.fr.g, L.fr.gm1, hi2);
                bool hi;
                const R sig = brems_lookup<R, false>(T, E.ct, e.g, e.gm1, hi).sig;
                const double x = coef * (double)sig * e.vrel * A.dt;
                if (settle(x, rng, L.dk, E.cell, kTagAccBr, kTagHiBr, rej, A.near_rel, Pej, L.near_br))
                    L.kind = kEvBr | ((A.proc & CMC_TRIDENT) ? kEvTrPending : 0u);
            }
            if ((A.proc & CMC_TRIDENT) && !L.kind) {
                const R sig = (R)phys::trident_sigma(T.Z, (double)e.g);
                if (sig > (R)0) {
                    const double x = coef * (double)sig * e.vrel * A.dt;
                    if (settle(x, rng, L.dk, E.cell, kTagAccTr, kTagHiTr, rej, A.near_rel, Pej, L.near_tr))
                        L.kind = kEvTr;
                }
            }
            L.reused = E.Ne < E.Ni && L.j + E.Ne < E.Ni;   // the electron pairs again later
        } else {
            const int64_t ig = E.g0 + L.mi;
            L.px = A.ph.px[ig]; L.py = A.ph.py[ig]; L.pz = A.ph.pz[ig]; L.Wm = A.ph.w[ig];
            L.fr = photon_frame(L.b, L.px, L.py, L.pz);
            bool hi2;
            bh_lookup<double>(T64, E.ct64, L.fr.g, L.ikd, L.wkd, hi2);
            const R k = L.b.mov ? (R)L.fr.g : photon_k<R>(L.px, L.py, L.pz);
            int ik; R wk; bool hi;
            const R sig = bh_lookup<R>(T, E.ct, k, ik, wk, hi);
            const double x = coef * (double)sig * photon_flux(L.fr, L.b) * A.dt;
            const double Pej = L.Wi / (L.Wm > L.Wi ? L.Wm : L.Wi);
            if (settle(x, rng, L.dk, E.cell, kTagAccBh, kTagHiBh, rej, A.near_rel, Pej, L.near_bh))
                L.kind = kEvBh;
            L.reused = E.Ng0 < E.Ni && L.j + E.Ng0 < E.Ni;
        }
    }
    return L;
}

// A wavefront settles the open pairs of a listed cell (ev_pair), one per
// lane in (pass, pair index) order, after ordering them in rec (kCandCap
// records of LDS).
template <typename R>
__device__ __forceinline__ EvLane<R> ev_settle(const StepArgs& A, const TabView<R>& T, const TabView<double>& T64,
                                               const Rng& rng, const EvCell<R>& E, uint64_t* rec, double rej) {
    const int lane = threadIdx.x & 63;
    const bool cand = lane < E.nc;
    // ---- the open pairs in (pass, pair index) order, one per lane
    {
        const bool has = lane < E.nc;
        const unsigned long long hb = __ballot(has);
        const uint32_t key = has ? ev_key(E.raw) : 0xFFFFFFFFu;
        int rank = 0;
        for (unsigned long long m = hb; m; m &= m - 1ull)
            rank += (uint32_t)__builtin_amdgcn_readlane((int)key, __ffsll((long long)m) - 1) < key;
        if (has) rec[rank] = E.raw;
        Team<64>::sync();
    }
    const uint64_t mine = cand ? rec[lane] : 0ull;
    return ev_pair<R>(A, T, T64, rng, E, mine, cand, rej);
}

// The kinematics of each lane's event: the energies sampled from the FP64
// tables (Sec. III.A), the mobile particle moved (L.px, L.py, L.pz), the
// products formed, the event's tallies (with the Trident test of a pair
// whose Bremsstrahlung was accepted, on the electron it left).  Lanes
// without an event do nothing.  Every lane of the wavefront calls it: with
// coop the wavefront inverts each CDF together (one round of table reads
// per event), else every lane bisects its own; both give the same abscissa.
struct EvKin {
    bool f_ph, f_tr, f_bh;
    double kx, ky, kz, pxm, pym, pzm, pxp, pyp, pzp;
    Tally t;
};

template <typename R>
__device__ __forceinline__ EvKin ev_kin(const StepArgs& A, const TabView<R>& T, const TabView<double>& T64,
                                           const Rng& rng, const EvCell<R>& E, EvLane<R>& L, bool coop) {
    const uint32_t evk = L.kind;
    Tally t = {};
    bool f_ph = false, f_tr = false, f_bh = false;
    double kx = 0, ky = 0, kz = 0, pxm = 0, pym = 0, pzm = 0, pxp = 0, pyp = 0, pzp = 0;
    const auto invert = [&](bool has, const CdfRow<double>& row, double xi, double& ct) {
        if (coop) return cdf_invert_wave<double>(has, row, E.ct64, xi, ct);
        return has ? cdf_invert<double>(row.T, row.kind, row.i, row.w, E.ct64, xi, ct) : 0.0;
    };
    // ---- first draw: Bremsstrahlung photon energy or Bethe-Heitler pair
    CdfRow<double> rowA = {};
    double xiA = 0.0;
    bool reqA = false;
    if (L.pass == 0 && (evk & kEvBr)) {
        const U4 q = rng.draw(L.dk, E.cell, kTagSmpBr);
        rowA = brems_row<double>(T64, L.BLd);
        xiA = u53(q.x, q.y);
        reqA = true;
    } else if (L.pass == 1 && (evk & kEvBh)) {
        const U4 q = rng.draw(L.dk, E.cell, kTagSmpBh);
        rowA = bh_row<double>(T64, L.ikd, L.wkd);
        xiA = u53(q.x, q.y);
        reqA = true;
    }
    double ctA = 0.0;
    const double tA = invert(reqA, rowA, xiA, ctA);
    bool tr = false;
    if (L.pass == 0 && evk) {
        if (evk & kEvBr) {
            double k, g2, g2m1;
            brems_energies(L.BLd.seg, L.fr.g, L.fr.gm1, ctA, k, g2, g2m1);
            const double pf = sqrt(g2m1 * (g2 + 1.0));
            lab_along(L.b, L.fr, k, k, kx, ky, kz);
            lab_along(L.b, L.fr, g2, pf, L.px, L.py, L.pz);
            t.ev_br++;
            t.E_br += L.Wm * sqrt(kx * kx + ky * ky + kz * kz);
            t.dE_el += L.Wm * lab_energy_change(L.b, L.fr, -k, g2, pf);
            t.W_br += L.Wm;
            f_ph = true;
        }
        tr = (evk & kEvTr) != 0;
        if (evk & kEvTrPending) {
            // Trident on the electron left by Bremsstrahlung (same pair)
            const double Pej = L.Wi / (L.Wm > L.Wi ? L.Wm : L.Wi);
            const Elec<R> e = L.b.mov ? electron_moving<R>(electron_frame(L.b, L.px, L.py, L.pz), L.b)
                                    : electron_p<R>(L.px, L.py, L.pz);
            const R sig = (R)phys::trident_sigma(T.Z, (double)e.g);
            if (sig > (R)0) {
                const double x = E.coef0 * (double)sig * e.vrel * A.dt;
                const double P = -expm1(-x);
                double U1, U2;
                accept_uniforms(rng, L.dk, E.cell, kTagAccTr, kTagHiTr, U1, U2);
                if (fabs(U1 - P) <= A.near_rel * P) t.near_tr++;
                tr = U1 < P && U2 < Pej;
            }
        }
    } else if (L.pass == 1 && evk) {
        double gpl, gmi;
        bh_energies(L.fr.g, tA, ctA, gpl, gmi);
        const double pplus = sqrt((gpl - 1.0) * (gpl + 1.0)), pminus = sqrt((gmi - 1.0) * (gmi + 1.0));
        lab_along(L.b, L.fr, gpl, pplus, pxp, pyp, pzp);
        lab_along(L.b, L.fr, gmi, pminus, pxm, pym, pzm);
        t.ev_bh++;
        t.E_bh += L.Wm * (sqrt(1.0 + pxp * pxp + pyp * pyp + pzp * pzp) + sqrt(1.0 + pxm * pxm + pym * pym + pzm * pzm));
        t.dE_ph += -L.Wm * L.fr.E;
        t.W_bh += L.Wm;
        f_bh = true;
    }
    // ---- Trident: pair energy, then the positron split
    U4 qt = {0u, 0u, 0u, 0u};
    CdfRow<double> rowB = {};
    Frame ft = {};   // the electron, after this pair's Bremsstrahlung, seen from the ion
    if (tr) {
        qt = rng.draw(L.dk, E.cell, kTagSmpTr);
        ft = electron_frame(L.b, L.px, L.py, L.pz);
        rowB = trident_row<double>(T64, ft.g);
    }
    double ctB = 0.0;
    const double tB = invert(tr, rowB, u53(qt.x, qt.y), ctB);
    double gpair = 0, gpl = 0, gmi = 0, gfm1 = 0;
    bool reqC = false;
    CdfRow<double> rowC = {};
    if (tr) {
        reqC = trident_pair(ft.gm1, tB, ctB, gpair, gpl, gmi, gfm1);
        if (reqC) rowC = split_row<double>(T64, gpair);
    }
    double ctC = 0.0;
    const double tC = invert(reqC, rowC, u53(qt.z, qt.w), ctC);
    if (reqC) split_energies(gpair, tC, ctC, gpl, gmi);
    if (tr) {
        const double gf = gfm1 + 1.0;
        const double pf = sqrt(gfm1 * (gf + 1.0));
        const double pplus = sqrt((gpl - 1.0) * (gpl + 1.0)), pminus = sqrt((gmi - 1.0) * (gmi + 1.0));
        lab_along(L.b, ft, gpl, pplus, pxp, pyp, pzp);
        lab_along(L.b, ft, gmi, pminus, pxm, pym, pzm);
        lab_along(L.b, ft, gf, pf, L.px, L.py, L.pz);
        t.ev_tr++;
        t.E_tr += L.Wm * (sqrt(1.0 + pxp * pxp + pyp * pyp + pzp * pzp) + sqrt(1.0 + pxm * pxm + pym * pym + pzm * pzm));
        t.dE_el += L.Wm * lab_energy_change(L.b, ft, -gpair, gf, pf);
        t.W_tr += L.Wm;
        f_tr = true;
    }
    return EvKin{f_ph, f_tr, f_bh, kx, ky, kz, pxm, pym, pzm, pxp, pyp, pzp, t};
}

// Tallies of a cell's pairs that ev_resolve settled beyond the lanes'
// records: near-threshold tests, and the pairs of converted photons after
// their conversion (counted by the pass, never tested).
struct ChainTally {
    int near_br, near_tr, near_bh;
    int bh_unpaired;
};

// rank of key among the lanes of mask (distinct keys)
__device__ __forceinline__ int key_rank(unsigned long long mask, uint32_t key) {
    int r = 0;
    for (unsigned long long m = mask; m; m &= m - 1ull)
        r += (uint32_t)__builtin_amdgcn_readlane((int)key, __ffsll((long long)m) - 1) < key;
    return r;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Events on particles that pair again later in their pass.  The pairs of
// a step are taken in order (Sec. III.A), so a particle's later pairs see
// it as its earlier events left it; the pass kernels tested every pair
// with the particles as the step found them.  Here, in one wavefront,
// each particle's first event stands and its later open pairs are
// dropped; then
//  - a converted photon pairs no more: its remaining pairs are not tested
//    (nor counted);
//  - an electron's remaining pairs are tested again, in order, with the
//    electron as each event leaves it (the cell's ions, at rest and of one
//    weight, are interchangeable, so the pair's ion does not matter): 64
//    pairs at a time, the first event found taking a free lane, and its
//    kinematics giving the electron's next state.
// The tests are those of ev_settle (FP64 P, the same draws keyed by the
// pair).  Returns false when an electron's pairs need testing again but
// the ions move or differ in weight, or when the lanes run out: the cell
// then takes the sequential step.  Every lane of the wavefront calls it.
template <typename R>
__device__ bool ev_resolve(const StepArgs& A, const TabView<R>& T, const TabView<double>& T64, const Rng& rng,
                           const EvCell<R>& E, EvLane<R>& L, double rej, ChainTally& X) {
    const int lane = threadIdx.x & 63;
    X = ChainTally{0, 0, 0, 0};
    if (!__ballot(L.kind != 0 && L.reused)) return true;
    // a particle's open pairs after its first event are dropped
    {
        const unsigned long long bev = __ballot(L.kind != 0);
        bool stale = false;
        for (unsigned long long m = bev; m; m &= m - 1ull) {
            const int o = __ffsll((long long)m) - 1;
            stale |= __builtin_amdgcn_readlane(L.pass, o) == L.pass && __builtin_amdgcn_readlane(L.mi, o) == L.mi &&
                     __builtin_amdgcn_readlane(L.j, o) < L.j;
        }
        if (stale) { L.kind = 0u; L.near_br = L.near_tr = L.near_bh = 0; }
    }
    const bool trig = L.kind != 0 && L.reused;
    // a converted photon's remaining pairs: of the pairs j = r + k N_g < N_i
    // of the photon of rank r, those after its conversion
    int unp = 0;
    if (trig && L.pass == 1) {
        const int Nm = E.Ng0, r = L.j % Nm, k = L.j / Nm;
        unp = (E.Ni - r + Nm - 1) / Nm - k - 1;
    }
    const unsigned long long chains = __ballot(trig && L.pass == 0);
    int nb_x = 0, nt_x = 0, nh_x = 0;
    bool ok = true;
    if (chains) {
        ok = (E.flg & kFlagIonsSame) != 0 && A.io.px == nullptr;
        // the lanes without an event are freed; their near counts are kept
        if (ok && L.kind == 0u) {
            nb_x += L.near_br; nt_x += L.near_tr; nh_x += L.near_bh;
            L.near_br = L.near_tr = L.near_bh = 0;
            L.pass = 2;
        }
        const int Nm = E.Ne, N = E.Ni;
        for (unsigned long long todo = ok ? chains : 0ull; todo && ok; todo &= todo - 1ull) {
            int tl = __ffsll((long long)todo) - 1;
            const int mi = __builtin_amdgcn_readlane(L.mi, tl);
            const double Wm = readlane_f64(L.Wm, tl), Wi = readlane_f64(L.Wi, tl);
            const double Pej = Wi / (Wm > Wi ? Wm : Wi);
            int jn = __builtin_amdgcn_readlane(L.j, tl) + Nm;    // the electron's next pair
            while (ok) {
                // the electron after the event on lane tl
                double px, py, pz;
                {
                    EvLane<R> Le = L;
                    if (lane != tl) Le.kind = 0u;
                    (void)ev_kin<R>(A, T, T64, rng, E, Le, true);
                    px = readlane_f64(Le.px, tl); py = readlane_f64(Le.py, tl); pz = readlane_f64(Le.pz, tl);
                }
                if (jn >= N) break;
                const Elec<R> e = electron_p<R>(px, py, pz);
                bool hi;
                const R sb = (A.proc & CMC_BREMS) ? brems_lookup<R, false>(T, E.ct, e.g, e.gm1, hi).sig : (R)0;
                const R st = (A.proc & CMC_TRIDENT) ? (R)phys::trident_sigma(T.Z, (double)e.g) : (R)0;
                const double xb = E.coef0 * (double)sb * e.vrel * A.dt;
                const double xt = E.coef0 * (double)st * e.vrel * A.dt;
                // the next pairs, 64 at a time, until one has an event
                int first = 64, jf = 0;
                uint32_t kf = 0u;
                int nbf = 0, ntf = 0;
                for (; jn < N; jn += 64 * Nm) {
                    const int jq = jn + lane * Nm;
                    const uint32_t dk = (uint32_t)(mi + (jq / Nm) * Nm);
                    int nb = 0, nt = 0;
                    uint32_t kind = 0u;
                    if (jq < N) {
                        if (sb > (R)0 && settle(xb, rng, dk, E.cell, kTagAccBr, kTagHiBr, rej, A.near_rel, Pej, nb))
                            kind = kEvBr | ((A.proc & CMC_TRIDENT) ? kEvTrPending : 0u);
                        if (!kind && st > (R)0 && settle(xt, rng, dk, E.cell, kTagAccTr, kTagHiTr, rej, A.near_rel, Pej, nt))
                            kind = kEvTr;
                    }
                    const unsigned long long bk = __ballot(kind != 0u);
                    first = bk ? __ffsll((long long)bk) - 1 : 64;
                    if (lane < first) { nb_x += nb; nt_x += nt; }   // tests that stand
                    if (bk) {
                        kf = (uint32_t)__builtin_amdgcn_readlane((int)kind, first);
                        nbf = __builtin_amdgcn_readlane(nb, first);
                        ntf = __builtin_amdgcn_readlane(nt, first);
                        jf = jn + first * Nm;
                        break;
                    }
                }
                if (first == 64) break;                   // no further event
                // the event takes a free lane
                const unsigned long long bfree = __ballot(L.kind == 0u);
                if (!bfree) { ok = false; break; }
                const int fl = __ffsll((long long)bfree) - 1;
                if (lane == fl) {
                    L.pass = 0; L.j = jf; L.mi = mi; L.ii = 0;
                    L.dk = (uint32_t)(mi + (jf / Nm) * Nm);
                    L.kind = kf;
                    L.near_br = nbf; L.near_tr = ntf; L.near_bh = 0;
                    L.px = px; L.py = py; L.pz = pz; L.Wm = Wm; L.Wi = Wi;
                    L.b = Ion{0.0, 0.0, 0.0, 1.0, false};
                    L.fr = electron_frame(L.b, px, py, pz);
                    if (kf & kEvBr) {
                        bool hi2;
                        L.BLd = brems_lookup<double, false>(T64, E.ct64, L.fr.g, L.fr.gm1, hi2);
                    }
                    L.reused = true;
                    L.last = true;
                }
                tl = fl;
                jn = jf + Nm;
            }
        }
    }
    if (!ok) return false;
    // the last event of each electron writes its momentum
    {
        const unsigned long long bev = __ballot(L.kind != 0u && L.pass == 0);
        bool later = false;
        for (unsigned long long m = bev; m; m &= m - 1ull) {
            const int o = __ffsll((long long)m) - 1;
            later |= __builtin_amdgcn_readlane(L.mi, o) == L.mi && __builtin_amdgcn_readlane(L.j, o) > L.j;
        }
        L.last = !later;
    }
    X.near_br = wave_sum_i32(nb_x);
    X.near_tr = wave_sum_i32(nt_x);
    X.near_bh = wave_sum_i32(nh_x);
    X.bh_unpaired = wave_sum_i32(unp);
    return true;
}

// The wavefront applies the settled events of its lanes: samples the
// energies in FP64, moves the mobile particles, writes the products at
// slots in (pass, pair index) order (ranks of the pair keys among the
// lanes), and writes the event tallies and the counts.  staged_all and
// n_conv: the workgroup kernel has every photon staged and removes n_conv
// converted ones beside this, so new photons go straight to their final
// slots.  X: the tallies of the pairs ev_resolve evaluated beyond the lanes.
template <typename R>
__device__ __forceinline__ void ev_apply(const StepArgs& A, const TabView<R>& T, const TabView<double>& T64,
                                         const Rng& rng, const EvCell<R>& E, EvLane<R>& L, bool staged_all,
                                         int n_conv, const ChainTally& X) {
    const int lane = threadIdx.x & 63;
    const int n = __popcll(__ballot(L.kind != 0));
    const EvKin K = ev_kin<R>(A, T, T64, rng, E, L, n <= 8);
    Tally t = K.t;
    t.near_br += L.near_br; t.near_tr += L.near_tr; t.near_bh += L.near_bh;
    const bool f_ph = K.f_ph, f_tr = K.f_tr, f_bh = K.f_bh;
    const double kx = K.kx, ky = K.ky, kz = K.kz, pxm = K.pxm, pym = K.pym, pzm = K.pzm;
    const double pxp = K.pxp, pyp = K.pyp, pzp = K.pzp;
    const int64_t par = L.pass == 0 ? E.e0 + L.mi : E.g0 + L.mi;
    if (L.pass == 0 && (f_ph || f_tr) && L.last) { A.el.px[par] = L.px; A.el.py[par] = L.py; A.el.pz[par] = L.pz; }
    // slots in (pass, pair) order: the rank of the lane's key among the
    // lanes with a product of the kind
    const unsigned long long b_ph = __ballot(f_ph), b_tr = __ballot(f_tr), b_bh = __ballot(f_bh);
    const int n_ph = __popcll(b_ph), n_tr = __popcll(b_tr), n_bh = __popcll(b_bh);
    const uint32_t key = ((uint32_t)L.pass << 16) | (uint32_t)L.j;
    const int r_ph = key_rank(b_ph, key), r_tr = key_rank(b_tr, key), r_bh = key_rank(b_bh, key);
    // with every photon staged the converted ones are removed beside
    // this: the new photons go straight to their final slots
    const int shift = staged_all ? n_conv : 0;
    if (f_ph) {
        const int slot = E.Ng0 + r_ph;
        if (slot < E.cap_ph) {
            const int64_t at = E.g0 + slot - shift;
            A.ph.px[at] = kx; A.ph.py[at] = ky; A.ph.pz[at] = kz; A.ph.w[at] = L.Wm;
            if (A.ph.parent) A.ph.parent[at] = par;
        } else t.drop_ph++;
    }
    if (f_tr || f_bh) {
        const int o = f_tr ? r_tr : n_tr + r_bh;
        if (E.cnt_ne0 + o < E.cap_ne) {
            const int64_t at = E.ne0 + E.cnt_ne0 + o;
            A.ne.px[at] = pxm; A.ne.py[at] = pym; A.ne.pz[at] = pzm; A.ne.w[at] = L.Wm;
            if (A.ne.parent) A.ne.parent[at] = par;
        } else t.drop_el++;
        if (E.cnt_np0 + o < E.cap_np) {
            const int64_t at = E.np0 + E.cnt_np0 + o;
            A.np.px[at] = pxp; A.np.py[at] = pyp; A.np.pz[at] = pzp; A.np.w[at] = L.Wm;
            if (A.np.parent) A.np.parent[at] = par;
        } else t.drop_po++;
    }
    const int ph_count = min(E.cap_ph, E.Ng0 + n_ph) - shift;
    // tallies of the events (the pair counts were written by the
    // passes).  A lane holds one open pair: each of its counts is 0 or
    // 1 (one event of a kind, one near-threshold test of a process,
    // one product of a kind), and only lanes with an event carry
    // energies and weights, which are added lane by lane in pair order.
    const auto count = [](long long v) { return (long long)__popcll(__ballot(v != 0)); };
    const long long iv[9] = {count(t.ev_br), count(t.ev_tr), count(t.ev_bh), count(t.near_br) + X.near_br,
                             count(t.near_tr) + X.near_tr, count(t.near_bh) + X.near_bh, count(t.drop_ph), count(t.drop_el),
                             count(t.drop_po)};
    double dv[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (unsigned long long m = __ballot(f_ph || f_tr || f_bh); m; m &= m - 1ull) {
        const int e = __ffsll((long long)m) - 1;
        dv[0] += lane_f64(t.E_br, e); dv[1] += lane_f64(t.E_tr, e); dv[2] += lane_f64(t.E_bh, e);
        dv[3] += lane_f64(t.dE_el, e); dv[4] += lane_f64(t.dE_ph, e);
        dv[5] += lane_f64(t.W_br, e); dv[6] += lane_f64(t.W_tr, e); dv[7] += lane_f64(t.W_bh, e);
    }
    if (lane == 0) {
        int64_t* ti = A.ti + E.c * CMC_NI;
        ti[CMC_I_EV_BR] = iv[0]; ti[CMC_I_EV_TR] = iv[1]; ti[CMC_I_EV_BH] = iv[2];
        ti[CMC_I_NEAR_BR] = iv[3]; ti[CMC_I_NEAR_TR] = iv[4]; ti[CMC_I_NEAR_BH] = iv[5];
        ti[CMC_I_DROP_PH] = iv[6]; ti[CMC_I_DROP_EL] = iv[7]; ti[CMC_I_DROP_PO] = iv[8];
        if (X.bh_unpaired) ti[CMC_I_PAIRS_BH] -= X.bh_unpaired;
        double* td = A.td + E.c * CMC_ND + CMC_D_E_BR;
        for (int q = 0; q < 8; ++q) td[q] = dv[q];
        if (A.ph.count && (!n_bh || staged_all)) A.ph.count[E.c] = ph_count;
        A.ne.count[E.c] = min(E.cap_ne, E.cnt_ne0 + n_tr + n_bh);
        A.np.count[E.c] = min(E.cap_np, E.cnt_np0 + n_tr + n_bh);
        if (iv[6] + iv[7] + iv[8]) atomicOr(A.status, CMC_ST_OVERFLOW);
    }
}

// One workgroup per listed cell.  Cells flagged by the pass kernels (more
// open pairs than kCandCap, more particles than the pass kernel's LDS) run
// the sequential step.  Otherwise the first wavefront settles the open
// pairs with P (same arithmetic as the pass kernels: lookups from the full
// tables give the same values as the slices); an event on a particle used
// by a later pair of its pass sends the cell to the sequential step too.
// Else it applies the events in (pass, pair) order: samples the energies,
// writes the products, and the four wavefronts then drop the converted
// photons.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_events(StepArgs A, TabView<R> T, TabView<double> T64, Work W,
                                                     int from_wave) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ CollideShared<R> sh;
    __shared__ uint64_t rec[kCandCap];
    __shared__ uint32_t killed[CMC_MAX_PER_CELL / 32];
    __shared__ int ctl[4];        // [0] sequential step, [1] photons converted, [2] first to move, [3] photon count
    __shared__ int wcnt[4][4];    // survivors per chunk group and wavefront
    __shared__ int kpre[kStagePh / 32];   // converted photons before each bitmap word
    const Smem S = carve(smem_raw, A.maxn);
    // staged photons (over S: an item takes either the sequential step or
    // the event path)
    double* const stx = reinterpret_cast<double*>(smem_raw);
    double* const sty = stx + kStagePh;
    double* const stz = sty + kStagePh;
    double* const stw = stz + kStagePh;
    int64_t* const stp = reinterpret_cast<int64_t*>(stw + kStagePh);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // the listed cells, or those the wavefront event kernel handed over
    const int32_t* list = from_wave ? W.list_wg : W.list_ev;
    const int n_items = W.counters[from_wave ? kCntWg : kCntEv];
    const double rej = 2.0 * (1.0 + A.near_rel);
    const Rng rng = step_rng(A);
    // the block's first cell is read beside the count (the list has
    // n_cells >= gridDim.x entries; an entry past the count is not used)
    int64_t c_next = list[blockIdx.x];
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t c = c_next;
        if (item + (int)gridDim.x < n_items) c_next = list[item + gridDim.x];
        const EvCell<R> E = ev_cell<R>(A, W, c, lane);
        const int64_t g0 = E.g0;
        const int Ng0 = E.Ng0, cap_ph = E.cap_ph;
        const bool slow = (E.flg & kFlagSlow) != 0;
        // ctl is read by the other wavefronts only after the barrier that
        // ends wavefront 0's work; wavefront 0 may set ctl[0..3] meanwhile
        if (threadIdx.x == 0) { ctl[0] = slow ? 1 : 0; ctl[1] = 0; }
        // while wavefront 0 settles the open pairs, the others copy the
        // cell's first photons to LDS (when a Bethe-Heitler pair is open):
        // the removal of converted photons then reads them from there
        const bool bh_open = __ballot(lane < E.nc && ev_pass(E.raw) == 1) != 0ull;
        const int n_st = (!slow && bh_open) ? min(Ng0, kStagePh) : 0;
        if (wv != 0 && n_st > 0) {
            constexpr int kPer = (kStagePh + kThreads - 65) / (kThreads - 64);
            double vx[kPer], vy[kPer], vz[kPer], vw[kPer];
            int64_t vp[kPer];
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                // clamped into the live photons: every load is issued at once
                const int64_t at = g0 + min((int)threadIdx.x - 64 + k * (kThreads - 64), n_st - 1);
                vx[k] = A.ph.px[at]; vy[k] = A.ph.py[at]; vz[k] = A.ph.pz[at]; vw[k] = A.ph.w[at];
                vp[k] = A.ph.parent ? A.ph.parent[at] : -1;
            }
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int a = (int)threadIdx.x - 64 + k * (kThreads - 64);
                if (a < n_st) { stx[a] = vx[k]; sty[a] = vy[k]; stz[a] = vz[k]; stw[a] = vw[k]; stp[a] = vp[k]; }
            }
        }
        // Wavefront 0 settles the open pairs; its lanes keep the pair's
        // particle, ion and FP64 lookup for the sampling after the barrier.
        EvLane<R> L{};
        ChainTally X{};
        // with every live photon staged, the survivors of a conversion are
        // moved by wavefronts 1-3 while wavefront 0 samples the events
        const bool staged_all = n_st == Ng0;
        if (wv == 0 && !slow) {
            L = ev_settle<R>(A, T, T64, rng, E, rec, rej);
            // events on particles that pair again later: resolved in order,
            // or (when that cannot be done here) the cell is redone by the
            // sequential step below
            if (!ev_resolve<R>(A, T, T64, rng, E, L, rej, X)) {
                if (lane == 0) ctl[0] = 1;
            } else {
                const int mi = L.mi;
                const bool conv = L.pass == 1 && (L.kind & kEvBh);
                const unsigned long long b_cv = __ballot(conv);
                if (b_cv) {
                    // converted photons: a bitmap, and for the staged case the
                    // count before each of its words
                    const int words = (Ng0 + 31) / 32;
                    for (int i = lane; i < words; i += 64) killed[i] = 0u;
                    Team<64>::sync();
                    if (conv) atomicOr(&killed[mi >> 5], 1u << (mi & 31));
                    Team<64>::sync();
                    if (staged_all) {
                        const int v = lane < words ? __popc(killed[lane]) : 0;
                        int incl = v;
#pragma unroll
                        for (int o = 1; o < 32; o <<= 1) {
                            const int y = __shfl_up(incl, o, 64);
                            if (lane >= o) incl += y;
                        }
                        if (lane < words) kpre[lane] = incl - v;
                    }
                    // photons before the first converted one stay where they are
                    int first = conv ? mi : 0x7FFFFFFF;
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) first = min(first, __shfl_xor(first, o, 64));
                    const int n_new = __popcll(__ballot(L.pass == 0 && (L.kind & kEvBr)));
                    if (lane == 0) { ctl[1] = __popcll(b_cv); ctl[2] = first; ctl[3] = min(cap_ph, Ng0 + n_new); }
                }
            }
        }
        __syncthreads();   // ctl, the bitmap and the staged photons
        if (ctl[0]) {
            collide_cell<R>(A, T, T64, rng, c, S, sh);
            __syncthreads();
            continue;
        }
        const int n_conv = ctl[1];
        if (wv == 0 && !slow) ev_apply<R>(A, T, T64, rng, E, L, staged_all, n_conv, X);
        if (wv != 0 && n_conv && staged_all) {
            // each survivor at or after the first converted photon moves down
            // by the converted photons before it, read from LDS: no photon is
            // read from global memory, so the moves need no ordering
            for (int a = ctl[2] + (int)threadIdx.x - 64; a < Ng0; a += kThreads - 64) {
                const uint32_t kw = killed[a >> 5];
                if ((kw >> (a & 31)) & 1u) continue;
                const int64_t dst = g0 + a - (kpre[a >> 5] + __popc(kw & ((1u << (a & 31)) - 1u)));
                A.ph.px[dst] = stx[a]; A.ph.py[dst] = sty[a]; A.ph.pz[dst] = stz[a]; A.ph.w[dst] = stw[a];
                if (A.ph.parent) A.ph.parent[dst] = stp[a];
            }
        }
        __syncthreads();
        if (n_conv && !staged_all) {
            // stable in-place removal of the converted photons: each
            // wavefront reads four chunks of 64 of a group of 1024 before any
            // is written (a survivor only moves down, never into a chunk not
            // yet read), the chunk counts give every survivor its slot
            const int end = ctl[3];
            const unsigned long long below = (1ull << lane) - 1ull;
            // one group; with every photon of it staged no global read is
            // made, so the wavefronts never wait for the product writes
            const auto group = [&](int base, int wpos, auto staged) {
                double vx[4], vy[4], vz[4], vw[4];
                int64_t pp[4];
                bool keep[4];
                unsigned long long bk[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = base + (4 * u + wv) * 64 + lane;
                    keep[u] = a < end && !(a < Ng0 && ((killed[a >> 5] >> (a & 31)) & 1u));
                    vx[u] = vy[u] = vz[u] = vw[u] = 0.0;
                    pp[u] = -1;
                    if (keep[u] && (decltype(staged)::value || a < n_st)) {
                        vx[u] = stx[a]; vy[u] = sty[a]; vz[u] = stz[a]; vw[u] = stw[a]; pp[u] = stp[a];
                    } else if (!decltype(staged)::value && keep[u]) {
                        vx[u] = A.ph.px[g0 + a]; vy[u] = A.ph.py[g0 + a]; vz[u] = A.ph.pz[g0 + a]; vw[u] = A.ph.w[g0 + a];
                        if (A.ph.parent) pp[u] = A.ph.parent[g0 + a];
                    }
                    bk[u] = __ballot(keep[u]);
                    if (lane == 0) wcnt[u][wv] = __popcll(bk[u]);
                }
                __syncthreads();
                int at = wpos;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int mine0 = at;
                    for (int w = 0; w < 4; ++w) { if (w < wv) mine0 += wcnt[u][w]; at += wcnt[u][w]; }
                    if (keep[u]) {
                        const int64_t dst = g0 + mine0 + __popcll(bk[u] & below);
                        A.ph.px[dst] = vx[u]; A.ph.py[dst] = vy[u]; A.ph.pz[dst] = vz[u]; A.ph.w[dst] = vw[u];
                        if (A.ph.parent) A.ph.parent[dst] = pp[u];
                    }
                }
                __syncthreads();
                return at;
            };
            int wpos = ctl[2] & ~63;
            for (int base = ctl[2] & ~63; base < end; base += 1024)
                wpos = (base + 1024 <= n_st || end <= n_st) ? group(base, wpos, std::true_type{})
                                                            : group(base, wpos, std::false_type{});
            if (threadIdx.x == 0 && A.ph.count) A.ph.count[c] = wpos;
        }
        __syncthreads();   // every read of ctl and of the LDS lists precedes the next cell
    }
}


// One lane per listed cell: the cells the stream kernel lists with at most
// kLaneCap open pairs, Trident off and both passes done by it (nearly
// every listed cell of the Bremsstrahlung workloads).  Its electrons pair
// once, so no event falls on an electron used by a later pair.  The lane
// settles the photon-ion pairs first: a conversion hands the cell to
// list_ev before anything is written (its converted photons need the
// workgroup kernel).  Then it settles the electron-ion pairs in pair order
// (ev_pair) and applies their events one after the other (ev_kin, each
// lane inverting its own CDFs): the values, product slots and tallies of
// the wavefront kernel, whose lanes take the same pairs in the same order
// and add the tallies in pair order.  Many cells are in flight at once
// where the wavefront kernel has one per wavefront.
template <typename R>
__global__ __launch_bounds__(kThreads, 2) void k_events_lane(StepArgs A, TabView<R> T, TabView<double> T64, Work W) {
    __shared__ uint64_t rec[kLaneCap][kThreads];   // per lane (column): its cell's open-pair records
    const int n_items = W.counters[kCntLane];
    const double rej = 2.0 * (1.0 + A.near_rel);
    const Rng rng = step_rng(A);
    for (int item = (int)(blockIdx.x * kThreads + threadIdx.x); item < n_items; item += (int)(gridDim.x * kThreads)) {
        const int64_t c = W.list_lane[item];
        const EvCell<R> E = ev_cell<R>(A, W, c, 0);
        bool hand = (E.flg & kFlagSlow) != 0 || E.ncr > kLaneCap || E.Ne < E.Ni || (A.proc & CMC_TRIDENT);
        const int nc = hand ? 0 : E.nc;
        // the cell's records in pair order, (pass, j), in the lane's column
        // of LDS (insertion sort: at most kLaneCap records)
        for (int i = 0; i < nc; ++i) {
            const uint64_t v = W.cand[c * kCandCap + i];
            int j = i;
            for (; j > 0 && ev_key(rec[j - 1][threadIdx.x]) > ev_key(v); --j) rec[j][threadIdx.x] = rec[j - 1][threadIdx.x];
            rec[j][threadIdx.x] = v;
        }
        // the photon-ion pairs: their near-threshold tests, or a conversion
        int near_bh = 0;
        for (int k = 0; k < nc && !hand; ++k) {
            const uint64_t rk = rec[k][threadIdx.x];
            if (ev_pass(rk) != 1) continue;
            const EvLane<R> L = ev_pair<R>(A, T, T64, rng, E, rk, true, rej);
            hand = L.kind != 0u;
            near_bh += L.near_bh != 0 ? 1 : 0;
        }
        if (hand) {
            W.list_ev[atomicAdd(&W.counters[kCntEv], 1)] = (int32_t)c;
            continue;
        }
        long long iv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        double dv[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        iv[5] = near_bh;
        int n_ph = 0;
        for (int k = 0; k < nc; ++k) {
            const uint64_t rk = rec[k][threadIdx.x];
            if (ev_pass(rk) != 0) continue;   // photon-ion pairs without an event: counted above
            EvLane<R> L = ev_pair<R>(A, T, T64, rng, E, rk, true, rej);
            const EvKin K = ev_kin<R>(A, T, T64, rng, E, L, false);
            Tally t = K.t;
            t.near_br += L.near_br; t.near_tr += L.near_tr; t.near_bh += L.near_bh;
            const int64_t par = E.e0 + L.mi;
            if ((K.f_ph || K.f_tr) && L.last) { A.el.px[par] = L.px; A.el.py[par] = L.py; A.el.pz[par] = L.pz; }
            if (K.f_ph) {
                const int slot = E.Ng0 + n_ph;
                if (slot < E.cap_ph) {
                    const int64_t at = E.g0 + slot;
                    A.ph.px[at] = K.kx; A.ph.py[at] = K.ky; A.ph.pz[at] = K.kz; A.ph.w[at] = L.Wm;
                    if (A.ph.parent) A.ph.parent[at] = par;
                } else t.drop_ph++;
                ++n_ph;
            }
            iv[0] += t.ev_br != 0; iv[1] += t.ev_tr != 0; iv[2] += t.ev_bh != 0;
            iv[3] += t.near_br != 0; iv[4] += t.near_tr != 0; iv[5] += t.near_bh != 0;
            iv[6] += t.drop_ph != 0; iv[7] += t.drop_el != 0; iv[8] += t.drop_po != 0;
            if (K.f_ph || K.f_tr || K.f_bh) {
                dv[0] += t.E_br; dv[1] += t.E_tr; dv[2] += t.E_bh; dv[3] += t.dE_el; dv[4] += t.dE_ph;
                dv[5] += t.W_br; dv[6] += t.W_tr; dv[7] += t.W_bh;
            }
        }
        int64_t* ti = A.ti + c * CMC_NI;
        ti[CMC_I_EV_BR] = iv[0]; ti[CMC_I_EV_TR] = iv[1]; ti[CMC_I_EV_BH] = iv[2];
        ti[CMC_I_NEAR_BR] = iv[3]; ti[CMC_I_NEAR_TR] = iv[4]; ti[CMC_I_NEAR_BH] = iv[5];
        ti[CMC_I_DROP_PH] = iv[6]; ti[CMC_I_DROP_EL] = iv[7]; ti[CMC_I_DROP_PO] = iv[8];
        double* td = A.td + c * CMC_ND + CMC_D_E_BR;
        for (int q = 0; q < 8; ++q) td[q] = dv[q];
        if (A.ph.count) A.ph.count[c] = min(E.cap_ph, E.Ng0 + n_ph);
        A.ne.count[c] = min(E.cap_ne, E.cnt_ne0);
        A.np.count[c] = min(E.cap_np, E.cnt_np0);
        if (iv[6] + iv[7] + iv[8]) atomicOr(A.status, CMC_ST_OVERFLOW);
    }
}

// One wavefront per listed cell, four cells per workgroup, no workgroup
// barrier and little LDS: a cell whose open pairs are all electron-ion
// pairs, none of whose events falls on an electron used by a later pair,
// is settled and applied here (the Bremsstrahlung workloads: nearly every
// listed cell).  Any other listed cell (the sequential step, open
// Bethe-Heitler pairs, whose converted photons need the workgroup's
// compaction) is handed to list_wg, which k_events walks next.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_events_wave(StepArgs A, TabView<R> T, TabView<double> T64, Work W) {
    __shared__ uint64_t rec[kWaves][kCandCap];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n_items = W.counters[kCntEv];
    const double rej = 2.0 * (1.0 + A.near_rel);
    const Rng rng = step_rng(A);
    for (int item = blockIdx.x * kWaves + wv; item < n_items; item += gridDim.x * kWaves) {
        const int64_t c = W.list_ev[item];
        const EvCell<R> E = ev_cell<R>(A, W, c, lane);
        bool hand = (E.flg & kFlagSlow) != 0 || __ballot(lane < E.nc && ev_pass(E.raw) == 1) != 0ull;
        EvLane<R> L{};
        ChainTally X{};
        if (!hand) {
            L = ev_settle<R>(A, T, T64, rng, E, rec[wv], rej);
            hand = !ev_resolve<R>(A, T, T64, rng, E, L, rej, X);
        }
        if (hand) {
            if (lane == 0) W.list_wg[atomicAdd(&W.counters[kCntWg], 1)] = (int32_t)c;
            continue;
        }
        ev_apply<R>(A, T, T64, rng, E, L, false, 0, X);
    }
}

// ------------------------------------------------------------------ pair_cells
struct PairArgs {
    const int64_t *a_off, *b_off, *pair_off, *cid;
    const int32_t *a_cnt, *b_cnt;
    const double *wa, *wb;
    int32_t *pa, *pb;
    double* nab;
    int64_t n_cells;
    Rng rng;
    uint32_t tag_a, tag_b;
    int maxn;
};

__global__ __launch_bounds__(kThreads) void k_pair(PairArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double redd[kWaves];
    __shared__ uint32_t redu[kWaves];
    const Smem S = carve(smem_raw, A.maxn);
    for (int64_t c = blockIdx.x; c < A.n_cells; c += gridDim.x) {
        const int ca = (int)(A.a_off[c + 1] - A.a_off[c]), cb = (int)(A.b_off[c + 1] - A.b_off[c]);
        const int na = A.a_cnt ? max(0, min(ca, A.a_cnt[c])) : ca;
        const int nb = A.b_cnt ? max(0, min(cb, A.b_cnt[c])) : cb;
        const int64_t po = A.pair_off[c];
        const int N = (na > 0 && nb > 0) ? (na > nb ? na : nb) : 0;
        if (na > A.maxn || nb > A.maxn || A.pair_off[c + 1] - po < N) {
            const int room = (int)min((int64_t)N, A.pair_off[c + 1] - po);
            for (int j = threadIdx.x; j < room; j += kThreads) { A.pa[po + j] = -1; A.pb[po + j] = -1; }
            if (A.nab && threadIdx.x == 0) A.nab[c] = 0.0;
            continue;
        }
        double part = 0.0;
        if (N > 0) {
            const uint32_t cell = cell_word(A.cid, c);
            key_order(na, cell, A.tag_a, A.rng, S.keys, S.pm, S.bcnt, redu);
            key_order(nb, cell, A.tag_b, A.rng, S.keys, S.pi, S.bcnt, redu);
            for (int j = threadIdx.x; j < N; j += kThreads) {
                const int a = S.pm[j % na], b = S.pi[j % nb];
                A.pa[po + j] = a; A.pb[po + j] = b;
                const double x = A.wa[A.a_off[c] + a], y = A.wb[A.b_off[c] + b];
                part += x < y ? x : y;
            }
        }
        const double s = block_sum(part, redd);
        if (A.nab && threadIdx.x == 0) A.nab[c] = s;
        __syncthreads();
    }
}

__global__ void k_step_bump(uint64_t* counter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter += 1;
}

int grid_for(int64_t n_cells) {
    const int64_t cap = 256 * 64;
    return (int)(n_cells < cap ? (n_cells > 0 ? n_cells : 1) : cap);
}

}  // namespace
}  // namespace cmc

using namespace cmc;

// ------------------------------------------------------------------ decision launch
// LDS of one team: a cell's pass is sorted in LDS when it needs an order
// (cap particles per species).  Wavefront teams are limited to kWaveCap so
// that several workgroups of four teams share a compute unit; workgroup
// teams run a first launch whose LDS leaves room for kMainWgs workgroups per
// compute unit (the streaming pass needs occupancy, not LDS), and the passes
// it defers (an order above its cap) run in a second launch sized for one.
constexpr int kWaveCap = 1024;
constexpr int kMainWgs = 6;
constexpr size_t kLdsMax = 160 * 1024;

static int team_cap(int team, int maxn, bool fp64, int wgs_per_cu = 1) {
    const int rb = fp64 ? 8 : 4;
    int cap = team == 64 ? std::min(maxn, kWaveCap) : maxn;
    const size_t static_lds = team == 64 ? 4608 : 2560;   // at least the pass kernel's static LDS
    while (cap > 64 && (size_t)wgs_per_cu * ((size_t)(256 / team) * ((team_bytes(cap, rb, team) + 15) / 16 * 16) + static_lds) > kLdsMax)
        cap -= 64;
    return cap;
}

// dynamic LDS above the default needs the function attribute; it is set
// outside stream capture (a captured step reuses what an eager step set)
static void lds_attr(const void* fn, size_t bytes, hipStream_t st) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(st, &cap);
    if (cap == hipStreamCaptureStatusNone)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// compute units of the current device (queried once per device)
static int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
    return n;
}

// at most `want` workgroups, and no more than the device holds at once
// (kernel with `threads` threads and `dshm` bytes of dynamic LDS)
static unsigned resident_grid(const void* kernel, int threads, size_t dshm, int64_t want) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, dshm) == hipSuccess && per_cu > 0)
        want = std::min<int64_t>(want, (int64_t)per_cu * device_cus());
    return (unsigned)std::max<int64_t>(1, want);
}

// Optional timing of the pair-test kernels of a step: the first launch
// records `start` when it begins (timestamped by the launch itself), and
// `stop` is recorded on the stream after the last launch.
struct PassTiming {
    hipEvent_t start, stop;
    bool first;
};

// one launch of the pass kernels: teams of kT over all cells of a size
// class (filter 1: up to fcap particles per species, 2: above, 0: all), or
// over the passes a first launch deferred (from_list)
struct PassLaunch {
    int cap, filter, fcap, slow_cap, from_list;
    int passes;         // bit 0: the electron-ion pass, bit 1: the photon-ion pass
    unsigned grid;
    size_t dshm;
};

template <typename R, int kT, bool kMov>
static void launch_pass_m(const StepArgs& A, const TabView<R>& T, const Work& W, const PassLaunch& L,
                          hipStream_t st, PassTiming* pt) {
    // the list of the cells the stream kernel left (from_list 3, ions at
    // rest) has an instantiation of its own
    const auto launch = [&](auto plain, auto rest) {
        const auto kernel = (!kMov && L.from_list == 3) ? rest : plain;
        lds_attr((const void*)kernel, L.dshm, st);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (pt) { e0 = pt->first ? pt->start : nullptr; pt->first = false; }
        // The launch over the cells the stream kernel left holds only the
        // workgroups that fit on the device at once: when it left none, each
        // returns after one read of the count, in one round.
        const unsigned grid = (!kMov && L.from_list == 3) ? resident_grid((const void*)kernel, 256, L.dshm, L.grid)
                                                          : L.grid;
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(256), (uint32_t)L.dshm, st, e0, e1, 0u, A, T, W, L.cap,
                              L.filter, L.fcap, L.slow_cap, L.from_list);
    };
    const bool ei = (L.passes & 1) && (A.proc & (CMC_BREMS | CMC_TRIDENT)) != 0;
    const bool gi = (L.passes & 2) && (A.proc & CMC_BH) != 0;
    if (ei && gi && L.from_list != 1) {
        launch(k_pass<R, kT, 2, kMov>, k_pass<R, kT, 2, kMov, !kMov>);
    } else {
        if (ei) launch(k_pass<R, kT, 0, kMov>, k_pass<R, kT, 0, kMov, !kMov>);
        if (gi) launch(k_pass<R, kT, 1, kMov>, k_pass<R, kT, 1, kMov, !kMov>);
    }
}

template <typename R, int kT>
static void launch_pass_t(const StepArgs& A, const TabView<R>& T, const Work& W, const PassLaunch& L,
                          hipStream_t st, PassTiming* pt) {
    if (A.io.px) launch_pass_m<R, kT, true>(A, T, W, L, st, pt);
    else launch_pass_m<R, kT, false>(A, T, W, L, st, pt);
}

static void launch_team(const StepArgs& A, const cmc_tables_s* t, const Work& W, bool fp64, int team, int cap,
                        int filter, int fcap, int slow_cap, int from_list, int64_t max_blocks, hipStream_t st,
                        PassTiming* pt, int passes = 3) {
    PassLaunch L;
    L.cap = cap; L.filter = filter; L.fcap = fcap; L.slow_cap = slow_cap; L.from_list = from_list;
    L.passes = passes;
    L.dshm = ((team_bytes(cap, fp64 ? 8 : 4, team) + 15) / 16 * 16) * (size_t)(256 / team);
    const int64_t units = team == 64 ? (A.n_cells + 3) / 4 : A.n_cells;
    L.grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(units, max_blocks));
    if (fp64) {
        if (team == 64) launch_pass_t<double, 64>(A, view64(t), W, L, st, pt);
        else launch_pass_t<double, 256>(A, view64(t), W, L, st, pt);
    } else {
        if (team == 64) launch_pass_t<float, 64>(A, view32(t), W, L, st, pt);
        else launch_pass_t<float, 256>(A, view32(t), W, L, st, pt);
    }
}

// Team shapes: 256 workgroups, 64 wavefronts, kHybrid wavefronts for the
// cells up to the wavefront capacity and workgroups for the larger ones,
// kQueue workgroups that take the cells from the cost-sorted work queue,
// kSplit workgroups for the electron-ion pass and then wavefronts for the
// photon-ion pass (each wavefront's LDS sized for kSplitCap photons: a few
// photons cycled against many ions need no more, and small teams keep many
// cells in flight; larger orders are deferred to the large-LDS launch).
constexpr int kHybrid = -1;
constexpr int kQueue = -2;
constexpr int kSplit = -3;
constexpr int kSplitCap = 256;

// the stream kernel over all cells (cells in index order, or the work
// queue), before the pass kernels: ions at rest and an electron-ion process
template <typename R>
static void launch_stream_r(const StepArgs& A, const TabView<R>& T, const Work& W, int scap, int from_list,
                            hipStream_t st, PassTiming* pt) {
    const size_t dshm = (size_t)scap * ((A.proc & CMC_TRIDENT) ? 8 : 4);
    const bool tri = (A.proc & CMC_TRIDENT) != 0, ph = (A.proc & CMC_BH) != 0;
    const auto kernel = tri ? (ph ? k_stream<R, true, true> : k_stream<R, true, false>)
                            : (ph ? k_stream<R, false, true> : k_stream<R, false, false>);
    lds_attr((const void*)kernel, dshm, st);
    const int64_t cap_blocks = from_list == 2 ? ((int64_t)1 << 20) : 256 * 64;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(A.n_cells, cap_blocks));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pt) { e0 = pt->first ? pt->start : nullptr; pt->first = false; }
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kStreamThreads), (uint32_t)dshm, st, e0, e1, 0u, A, T, W, scap,
                          from_list);
}

// true when it ran: the pass kernels then walk the cells it left (from_list 3)
static bool launch_stream(const StepArgs& A, const cmc_tables_s* t, const Work& W, bool fp64, int big, int from_list,
                          hipStream_t st, PassTiming* pt) {
    if (A.io.px || !(A.proc & (CMC_BREMS | CMC_TRIDENT))) return false;
    const int scap = std::min(std::min(kStreamCap, A.maxn), big);
    if (scap <= 1024) return false;
    if (fp64) launch_stream_r<double>(A, view64(t), W, scap, from_list, st, pt);
    else launch_stream_r<float>(A, view32(t), W, scap, from_list, st, pt);
    return true;
}

// A launch plan of the pair tests: the team shape, and whether the stream
// kernel runs first
struct Plan {
    int team;
    bool stream;
};

static cmc_status launch_passes(const StepArgs& A, const cmc_tables_s* t, const Work& W, bool fp64, Plan plan,
                                hipStream_t st, PassTiming* pt = nullptr) {
    const int shape = plan.team;
    const auto launch_stream = [&](int from_list) {
        return plan.stream && ::launch_stream(A, t, W, fp64, team_cap(256, A.maxn, fp64, 1), from_list, st, pt);
    };
    const int big = team_cap(256, A.maxn, fp64, 1);
    const int main = std::min(big, team_cap(256, A.maxn, fp64, kMainWgs));
    const int small = team_cap(64, A.maxn, fp64);
    if (shape == 64) {
        // wavefront teams only: cells above their capacity take the sequential step
        launch_team(A, t, W, fp64, 64, small, 0, 0, small, 0, 256 * 64, st, pt);
    } else if (shape == kSplit) {
        // the stream kernel, then wavefront teams for the passes it left,
        // one launch per pass (the fused wavefront kernel holds too many
        // registers for the occupancy the photon-ion pass needs)
        const int sc = std::min(big, kSplitCap);
        const int fl = launch_stream(0) ? 3 : 0;
        launch_team(A, t, W, fp64, 64, sc, 0, 0, big, fl, 256 * 64, st, pt, 1);
        launch_team(A, t, W, fp64, 64, sc, 0, 0, big, fl, 256 * 64, st, pt, 2);
        if (big > sc) launch_team(A, t, W, fp64, 256, big, 0, 0, big, 1, 1024, st, pt);
    } else if (shape == kQueue) {
        // the cells sorted by cost, then one launch of a workgroup per queue
        // entry (up to 2^20 workgroups; beyond, each strides over the queue);
        // after the stream kernel, the cells it left (listed in about the
        // order it took them from the queue)
        hipLaunchKernelGGL(k_queue, dim3(1), dim3(kQThreads), 0, st, A, W);
        const int fl = launch_stream(2) ? 3 : 2;
        launch_team(A, t, W, fp64, 256, main, 0, 0, big, fl, (int64_t)1 << 20, st, pt);
        if (big > main) launch_team(A, t, W, fp64, 256, big, 0, 0, big, 1, 1024, st, pt);
    } else {
        const int fl = launch_stream(0) ? 3 : 0;
        if (shape == kHybrid) {
            launch_team(A, t, W, fp64, 64, small, 1, small, big, fl, 256 * 64, st, pt);
            launch_team(A, t, W, fp64, 256, main, 2, small, big, fl, 256 * 64, st, pt);
        } else {
            launch_team(A, t, W, fp64, 256, main, 0, 0, big, fl, 256 * 64, st, pt);
        }
        // the passes that needed more LDS than the first launch has
        if (big > main) launch_team(A, t, W, fp64, 256, big, 0, 0, big, 1, 1024, st, pt);
    }
    CMC_CHECK_LAUNCH("cmc_collide_step: k_pass");
    return CMC_OK;
}

// Autotuner of the pair-test launches: on the first step of a launch shape
// (device, cells, max_per_cell, processes, precision, moving ions, stream
// kernel allowed) each plan (team shape, with or without the stream kernel)
// is timed on that step's own cells (the pass kernels leave the particles
// untouched; the cell state is cleared before each plan and again
// afterwards) and the fastest is kept for the process.  The host waits for
// the timing once per launch shape.
struct TuneKey {
    int dev;
    int64_t n_cells;
    int maxn, proc, precision, moving, no_stream;
    bool operator<(const TuneKey& o) const {
        return std::tie(dev, n_cells, maxn, proc, precision, moving, no_stream) <
               std::tie(o.dev, o.n_cells, o.maxn, o.proc, o.precision, o.moving, o.no_stream);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, Plan> g_tune;

static bool tune_lookup(const TuneKey& k, Plan& plan) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    plan = it->second;
    return true;
}

static void tune_store(const TuneKey& k, Plan plan) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[k] = plan;
}

// reset() clears the cells' flags and counters (the cell-state launch)
// before each plan is timed: flags one plan sets (passes done by the
// stream kernel) would let another skip work.
template <typename Reset>
static cmc_status tune_passes(const StepArgs& A, const cmc_tables_s* t, const Work& W, bool fp64, hipStream_t st,
                              bool allow_stream, Plan& best, const Reset& reset) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) { set_error("cmc_collide_step: hipEventCreate failed"); return CMC_EDEVICE; }
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error("cmc_collide_step: hipEventCreate failed");
        return CMC_EDEVICE;
    }
    float best_ms = 0.0f;
    cmc_status rc = CMC_OK;
    const int other = A.maxn <= team_cap(64, A.maxn, fp64) ? 64 : kHybrid;
    const bool both = (A.proc & (CMC_BREMS | CMC_TRIDENT)) && (A.proc & CMC_BH);
    // the stream kernel applies to ions at rest with an electron-ion process
    const bool sk = allow_stream && !A.io.px && (A.proc & (CMC_BREMS | CMC_TRIDENT));
    Plan plans[6];
    int np = 0;
    plans[np++] = Plan{256, sk};            // the reference: workgroup teams
    if (sk) plans[np++] = Plan{256, false};
    plans[np++] = Plan{other, sk && other != 64};
    plans[np++] = Plan{kQueue, false};
    if (sk) plans[np++] = Plan{kQueue, true};
    if (both) plans[np++] = Plan{kSplit, sk};
    best = plans[0];
    for (int i = 0; i < np; ++i) {
        const Plan p = plans[i];
        reset();
        if ((rc = launch_passes(A, t, W, fp64, p, st)) != CMC_OK) break;   // warm-up
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 3 && rc == CMC_OK; ++r) rc = launch_passes(A, t, W, fp64, p, st);
        (void)hipEventRecord(e1, st);
        if (rc != CMC_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) { set_error("cmc_collide_step: timing failed"); rc = CMC_EDEVICE; break; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        // another plan must beat the reference by 3% (timing noise of a
        // few runs would otherwise pick a slower plan now and then)
        if (i == 0 || ms < best_ms * (i > 0 && best.team == plans[0].team && best.stream == plans[0].stream
                                          ? 0.97f : 1.0f)) {
            best_ms = ms;
            best = p;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

extern "C" size_t cmc_step_workspace_bytes(int64_t n_cells, int32_t schedule) {
    if (n_cells <= 0 || (schedule & ~CMC_SCHED_NO_STREAM) == CMC_SCHED_CELL) return 0;
    return work_bytes(n_cells);
}

static cmc_status set_species(SpeciesDev& d, const cmc_species* s, const char* name, bool need_count,
                              bool need_mom) {
    CMC_REQUIRE(s && s->off && s->w, CMC_EINVAL, "cmc_collide_step: %s: off and w are required", name);
    CMC_REQUIRE(!need_count || s->count, CMC_EINVAL, "cmc_collide_step: %s: count is required", name);
    CMC_REQUIRE(!need_mom || (s->px && s->py && s->pz), CMC_EINVAL,
                "cmc_collide_step: %s: px, py, pz are required", name);
    CMC_REQUIRE(aligned_to<int64_t>(s->off) && aligned_to<int32_t>(s->count) && aligned_to<double>(s->px) &&
                    aligned_to<double>(s->py) && aligned_to<double>(s->pz) && aligned_to<double>(s->w) &&
                    aligned_to<int64_t>(s->parent),
                CMC_EINVAL, "cmc_collide_step: %s: an array is not aligned to its element type", name);
    d.off = s->off; d.count = s->count; d.px = s->px; d.py = s->py; d.pz = s->pz; d.w = s->w;
    d.parent = s->parent;
    return CMC_OK;
}

// The step behind both entry points.  may_time: an untuned automatic
// schedule may time the team shapes on this call (else workgroup teams).
static cmc_status collide_step_impl(const char* who, cmc_tables t, const cmc_cells* cells, cmc_species* electrons,
                                    cmc_species* photons, const cmc_species* ions, cmc_species* new_el,
                                    cmc_species* new_po, const cmc_step_params* P, cmc_tallies* tal,
                                    void* workspace, size_t workspace_bytes, void* stream, bool may_time) {
    CMC_REQUIRE(t && cells && P && tal, CMC_EINVAL, "%s: NULL argument", who);
    CMC_REQUIRE(cells->n_cells >= 0 && cells->Zstar && cells->n_i && cells->T_e, CMC_EINVAL,
                "%s: cells incomplete", who);
    CMC_REQUIRE(tal->ti && tal->td && tal->status, CMC_EINVAL, "%s: tallies incomplete", who);
    CMC_REQUIRE(aligned_to<double>(cells->Zstar) && aligned_to<double>(cells->n_i) && aligned_to<double>(cells->T_e) &&
                    aligned_to<int64_t>(cells->cell_id) && aligned_to<int64_t>(tal->ti) && aligned_to<double>(tal->td) &&
                    aligned_to<int32_t>(tal->status) && aligned_to<uint64_t>(P->step_counter) &&
                    aligned_to<uint64_t>(workspace),
                CMC_EINVAL, "%s: a cell, tally, counter or workspace array is not aligned to its element type", who);
    CMC_REQUIRE(P->dt > 0.0, CMC_EINVAL, "%s: dt must be > 0", who);
    CMC_REQUIRE((P->processes & ~7u) == 0, CMC_EINVAL, "%s: unknown process bits", who);
    CMC_REQUIRE(P->precision == CMC_FP64 || P->precision == CMC_FP32, CMC_EINVAL,
                "%s: unknown precision %d", who, P->precision);
    CMC_REQUIRE((P->schedule & ~CMC_SCHED_NO_STREAM) >= 0 && (P->schedule & ~CMC_SCHED_NO_STREAM) <= 6, CMC_EINVAL,
                "%s: unknown schedule", who);
    CMC_REQUIRE(P->max_per_cell >= 1 && P->max_per_cell <= CMC_MAX_PER_CELL, CMC_ERANGE,
                "%s: max_per_cell = %d outside [1, %d]", who, P->max_per_cell, CMC_MAX_PER_CELL);
    CMC_REQUIRE(P->near_rel >= 0.0 && P->near_rel <= 1.0, CMC_EINVAL, "%s: near_rel outside [0, 1]", who);
    StepArgs A{};
    cmc_status s;
    if ((s = set_species(A.el, electrons, "electrons", false, true)) != CMC_OK) return s;
    if ((s = set_species(A.ph, photons, "photons", true, true)) != CMC_OK) return s;
    if ((s = set_species(A.io, ions, "ions", false, false)) != CMC_OK) return s;
    CMC_REQUIRE((!ions->px && !ions->py && !ions->pz) || (ions->px && ions->py && ions->pz), CMC_EINVAL,
                "%s: ions: px, py, pz must be all set (moving) or all NULL (at rest)", who);
    if ((s = set_species(A.ne, new_el, "new_el", true, true)) != CMC_OK) return s;
    if ((s = set_species(A.np, new_po, "new_po", true, true)) != CMC_OK) return s;
    A.Zs = cells->Zstar; A.ni = cells->n_i; A.Te = cells->T_e; A.cid = cells->cell_id;
    A.n_cells = cells->n_cells;
    A.dt = P->dt; A.near_rel = P->near_rel;
    A.rng.k0 = (uint32_t)P->seed; A.rng.k1 = (uint32_t)(P->seed >> 32);
    A.rng.step_lo = (uint32_t)P->step; A.rng.step_hi = (uint32_t)(P->step >> 32);
    A.proc = P->processes;
    A.maxn = P->max_per_cell;
    A.ti = tal->ti; A.td = tal->td; A.status = tal->status;
    if (A.n_cells == 0) return CMC_OK;
    hipStream_t st = as_stream(stream);
    const size_t shm = smem_bytes(A.maxn);
    const int grid = grid_for(A.n_cells);
    const bool fp64 = P->precision == CMC_FP64;
    if ((P->schedule & ~CMC_SCHED_NO_STREAM) == CMC_SCHED_CELL) {
        // one sequential workgroup per cell for every cell
        A.list = nullptr; A.list_n = nullptr;
        A.step_dev = P->step_counter;
        if (fp64) {
            lds_attr((const void*)k_collide<double>, shm, st);
            hipLaunchKernelGGL(k_collide<double>, dim3(grid), dim3(kThreads), shm, st, A, view64(t), view64(t));
        } else {
            lds_attr((const void*)k_collide<float>, shm, st);
            hipLaunchKernelGGL(k_collide<float>, dim3(grid), dim3(kThreads), shm, st, A, view32(t), view64(t));
        }
        CMC_CHECK_LAUNCH(who);
        if (P->step_counter) {
            hipLaunchKernelGGL(k_step_bump, dim3(1), dim3(64), 0, st, P->step_counter);
            CMC_CHECK_LAUNCH2(who, "step counter");
        }
        return CMC_OK;
    }
    const size_t need = work_bytes(A.n_cells);
    CMC_REQUIRE(workspace != nullptr && workspace_bytes >= need, CMC_EINVAL,
                "%s: workspace of %zu bytes required (got %zu)", who, need, workspace_bytes);
    const Work W = carve_work(workspace, A.n_cells);
    A.step_dev = W.step;
    const auto cell_state = [&](int advance) {
        hipLaunchKernelGGL(k_cell_state, dim3((unsigned)std::min<int64_t>((A.n_cells + 63) / 64, 4096)), dim3(64),
                           0, st, A.Zs, A.ni, A.Te, A.n_cells, (double)t->Z, t->ax, W, A.ti, A.td, A.status,
                           P->step_counter, P->step, advance);
    };
    const int sched = P->schedule & ~CMC_SCHED_NO_STREAM;
    const bool allow_stream = !(P->schedule & CMC_SCHED_NO_STREAM);
    Plan plan{sched == CMC_SCHED_WAVE ? 64
              : sched == CMC_SCHED_HYBRID ? kHybrid
              : sched == CMC_SCHED_QUEUE ? kQueue
              : sched == CMC_SCHED_SPLIT ? kSplit : 256, allow_stream};
    bool tuned = sched != CMC_SCHED_AUTO;
    TuneKey key{};
    if (!tuned) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        key = TuneKey{dev, A.n_cells, A.maxn, (int)A.proc, P->precision, A.io.px ? 1 : 0, allow_stream ? 0 : 1};
        tuned = tune_lookup(key, plan);
    }
    // the counter advances once, in the last cell-state launch of the step
    cell_state(tuned ? 1 : 0);
    CMC_CHECK_LAUNCH2(who, "k_cell_state");
    if (!tuned) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        (void)hipStreamIsCapturing(st, &cap);
        if (cap == hipStreamCaptureStatusNone && may_time) {
            cmc_status s2 = tune_passes(A, t, W, fp64, st, allow_stream, plan, [&]() { cell_state(0); });
            if (s2 != CMC_OK) return s2;
            tune_store(key, plan);
        } else {
            plan = Plan{256, allow_stream};   // no timing under graph capture: workgroup teams
        }
        cell_state(1);          // the timing runs filled the cell lists
        CMC_CHECK_LAUNCH2(who, "k_cell_state");
    }
    PassTiming timing{static_cast<hipEvent_t>(P->pass_events[0]), static_cast<hipEvent_t>(P->pass_events[1]), true};
    const bool timed = P->pass_events[0] && P->pass_events[1];
    cmc_status s1 = launch_passes(A, t, W, fp64, plan, st, timed ? &timing : nullptr);
    if (s1 != CMC_OK) return s1;
    if (timed && hipEventRecord(timing.stop, st) != hipSuccess) {
        set_error("%s: hipEventRecord of pass_events[1] failed", who);
        return CMC_EDEVICE;
    }
    // the listed cells: open pairs and events, or the sequential step (a
    // short list: a small grid)
    // When electron-ion pairs can be open, a wavefront per listed cell
    // first settles and applies the cells that need no workgroup and hands
    // the others on; with Bethe-Heitler alone every listed cell needs the
    // workgroup kernel, which then walks the list itself.
    // The event kernels walk their lists with as many workgroups as the
    // device holds at once (an empty or short list then costs one round)
    const size_t shm_ev = std::max(shm, (size_t)kStagePh * 40);
    const void* kev = fp64 ? (const void*)k_events<double> : (const void*)k_events<float>;
    lds_attr(kev, shm_ev, st);   // before the occupancy query, which sees the attribute
    const unsigned gev = resident_grid(kev, kThreads, shm_ev, std::min<int64_t>(A.n_cells, 512));
    const int from_wave = (A.proc & (CMC_BREMS | CMC_TRIDENT)) ? 1 : 0;
    if (from_wave && plan.stream && !(A.proc & CMC_TRIDENT)) {
        // the cells the stream kernel listed for a lane each (any it hands
        // back join list_ev before the wavefront kernel reads its length)
        const unsigned gl = (unsigned)std::min<int64_t>((A.n_cells + kThreads - 1) / kThreads, 2048);
        if (fp64) hipLaunchKernelGGL(k_events_lane<double>, dim3(gl), dim3(kThreads), 0, st, A, view64(t), view64(t), W);
        else hipLaunchKernelGGL(k_events_lane<float>, dim3(gl), dim3(kThreads), 0, st, A, view32(t), view64(t), W);
        CMC_CHECK_LAUNCH2(who, "k_events_lane");
    }
    if (from_wave) {
        const unsigned gw = resident_grid(fp64 ? (const void*)k_events_wave<double> : (const void*)k_events_wave<float>,
                                          kThreads, 0, std::min<int64_t>((A.n_cells + kWaves - 1) / kWaves, 2048));
        if (fp64) hipLaunchKernelGGL(k_events_wave<double>, dim3(gw), dim3(kThreads), 0, st, A, view64(t), view64(t), W);
        else hipLaunchKernelGGL(k_events_wave<float>, dim3(gw), dim3(kThreads), 0, st, A, view32(t), view64(t), W);
        CMC_CHECK_LAUNCH2(who, "k_events_wave");
    }
    if (fp64) hipLaunchKernelGGL(k_events<double>, dim3(gev), dim3(kThreads), shm_ev, st, A, view64(t), view64(t), W,
                                 from_wave);
    else hipLaunchKernelGGL(k_events<float>, dim3(gev), dim3(kThreads), shm_ev, st, A, view32(t), view64(t), W,
                            from_wave);
    CMC_CHECK_LAUNCH2(who, "k_events");
    return CMC_OK;
}

extern "C" cmc_status cmc_collide_step(cmc_tables t, const cmc_cells* cells, cmc_species* electrons,
                                       cmc_species* photons, const cmc_species* ions,
                                       cmc_species* new_el, cmc_species* new_po,
                                       const cmc_step_params* P, cmc_tallies* tal,
                                       void* workspace, size_t workspace_bytes, void* stream) {
    return collide_step_impl("cmc_collide_step", t, cells, electrons, photons, ions, new_el, new_po, P, tal,
                             workspace, workspace_bytes, stream, true);
}

// ------------------------------------------------------------------ no-allocation entry point
// The workspace of cmc_collide_step_noalloc, for callers that cannot
// allocate: a file-scope device array, one copy on every GPU the library
// runs on, held until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: the device address of each GPU's
// copy is taken once per device (hipGetSymbolAddress, with that device
// current) and only that address reaches the kernels.
constexpr int64_t kNoallocCells = 16384;
constexpr size_t kNoallocBytes = work_bytes(kNoallocCells);
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;   // device -> address of its `scratch`

static cmc_status scratch_of_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("cmc_collide_step_noalloc: hipGetDevice failed");
        return CMC_EDEVICE;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("cmc_collide_step_noalloc: hipGetSymbolAddress failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return CMC_EDEVICE;
        }
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return CMC_OK;
}

extern "C" size_t cmc_noalloc_max_cells(void) { return (size_t)kNoallocCells; }

extern "C" cmc_status cmc_collide_step_noalloc(cmc_tables t, const cmc_cells* cells, cmc_species* electrons,
                                               cmc_species* photons, const cmc_species* ions,
                                               cmc_species* new_el, cmc_species* new_po,
                                               const cmc_step_params* P, cmc_tallies* tal, void* stream) {
    CMC_REQUIRE(cells && P, CMC_EINVAL, "cmc_collide_step_noalloc: NULL argument");
    CMC_REQUIRE(cells->n_cells <= kNoallocCells, CMC_ERANGE,
                "cmc_collide_step_noalloc: %lld cells, above the %lld its static workspace holds",
                (long long)cells->n_cells, (long long)kNoallocCells);
    void* ws = nullptr;
    if (cells->n_cells > 0 && P->schedule != CMC_SCHED_CELL) {
        const cmc_status s = scratch_of_current_device(&ws);
        if (s != CMC_OK) return s;
    }
    return collide_step_impl("cmc_collide_step_noalloc", t, cells, electrons, photons, ions, new_el, new_po, P, tal,
                             ws, kNoallocBytes, stream, false);
}

extern "C" cmc_status cmc_pair_cells(int64_t n_cells, const int64_t* cell_id, const int64_t* a_off, const int32_t* a_cnt,
                                     const int64_t* b_off, const int32_t* b_cnt, const double* wa,
                                     const double* wb, uint64_t seed, uint64_t step, uint32_t pass,
                                     const int64_t* pair_off, int32_t* pa, int32_t* pb, double* n_ab,
                                     void* stream) {
    CMC_REQUIRE(n_cells >= 0, CMC_EINVAL, "cmc_pair_cells: n_cells < 0");
    CMC_REQUIRE(a_off && b_off && wa && wb && pair_off && pa && pb, CMC_EINVAL, "cmc_pair_cells: NULL argument");
    CMC_REQUIRE(aligned_to<int64_t>(cell_id) && aligned_to<int64_t>(a_off) && aligned_to<int64_t>(b_off) &&
                    aligned_to<int32_t>(a_cnt) && aligned_to<int32_t>(b_cnt) && aligned_to<double>(wa) &&
                    aligned_to<double>(wb) && aligned_to<int64_t>(pair_off) && aligned_to<int32_t>(pa) &&
                    aligned_to<int32_t>(pb) && aligned_to<double>(n_ab),
                CMC_EINVAL, "cmc_pair_cells: an array is not aligned to its element type");
    CMC_REQUIRE(pass == 1 || pass == 2, CMC_EINVAL, "cmc_pair_cells: pass must be 1 or 2");
    if (n_cells == 0) return CMC_OK;
    PairArgs A{};
    A.a_off = a_off; A.b_off = b_off; A.pair_off = pair_off; A.cid = cell_id; A.a_cnt = a_cnt; A.b_cnt = b_cnt;
    A.wa = wa; A.wb = wb; A.pa = pa; A.pb = pb; A.nab = n_ab; A.n_cells = n_cells;
    A.rng.k0 = (uint32_t)seed; A.rng.k1 = (uint32_t)(seed >> 32);
    A.rng.step_lo = (uint32_t)step; A.rng.step_hi = (uint32_t)(step >> 32);
    A.tag_a = pass == 1 ? kTagKeyE : kTagKeyG;
    A.tag_b = pass == 1 ? kTagKeyIE : kTagKeyIG;
    A.maxn = CMC_MAX_PER_CELL;
    const size_t shm = smem_bytes(A.maxn);
    (void)hipFuncSetAttribute((const void*)k_pair, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k_pair, dim3(grid_for(n_cells)), dim3(kThreads), shm, as_stream(stream), A);
    CMC_CHECK_LAUNCH("cmc_pair_cells");
    return CMC_OK;
}
