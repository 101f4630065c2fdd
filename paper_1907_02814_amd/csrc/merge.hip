// merge.hip -- the step after: products join their populations, and a
// population gets new slabs.  Created particles are macro-particles of their
// species (Sec. III.A): the photons one step creates convert in the next,
// and the electrons and positrons of a pair radiate and make pairs in turn
// (the chains of Sec. IV).  A step appends its photons to the photon
// population itself; cmc_merge_species appends a product buffer (new
// electrons, new positrons) to a population cell by cell, and
// cmc_rebin_offsets / cmc_rebin_copy lay a population out again with room
// in every cell.  Pure data movement: one wavefront per cell, coalesced
// copies of the structure-of-arrays records.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace cmc {
namespace {

constexpr int kThreads = 256;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 16;      // consecutive cells per thread and round of the offsets scan

struct Sp {
    const int64_t* off;
    int32_t* count;
    double *px, *py, *pz, *w;
    int64_t* parent;
};

__device__ __forceinline__ int live_of(const int64_t* off, const int32_t* count, int64_t c) {
    const int64_t cap = off[c + 1] - off[c];
    if (!count) return (int)cap;
    const int64_t n = count[c];
    return (int)(n < 0 ? 0 : (n < cap ? n : cap));
}

__device__ __forceinline__ void copy_rec(const Sp& d, int64_t b, const Sp& s, int64_t a) {
    if (d.px) { d.px[b] = s.px[a]; d.py[b] = s.py[a]; d.pz[b] = s.pz[a]; }
    d.w[b] = s.w[a];
    if (d.parent && s.parent) d.parent[b] = s.parent[a];
}

// one wavefront per cell: src's live records after dst's, as far as dst's
// slab holds them, in src's order; src emptied
__global__ __launch_bounds__(kThreads) void k_merge(Sp d, Sp s, int64_t n, int64_t* dropped, int32_t* status) {
    const int lane = threadIdx.x & 63;
    for (int64_t c = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); c < n;
         c += (int64_t)gridDim.x * (kThreads / 64)) {
        const int nd = live_of(d.off, d.count, c), ns = live_of(s.off, s.count, c);
        const int room = (int)(d.off[c + 1] - d.off[c]) - nd;
        const int nk = ns < room ? ns : room;
        const int64_t a0 = s.off[c], b0 = d.off[c] + nd;
        for (int i = lane; i < nk; i += 64) copy_rec(d, b0 + i, s, a0 + i);
        if (lane == 0) {
            d.count[c] = nd + nk;
            s.count[c] = 0;
            if (dropped) dropped[c] = ns - nk;
            if (ns > nk && status) atomicOr(status, CMC_ST_OVERFLOW);
        }
    }
}

// off_new[c + 1] = off_new[c] + live(c) + headroom: one workgroup, rounds of
// kScanThreads x kScanItems cells (each thread scans its consecutive cells,
// the workgroup scans the thread totals, a running carry joins the rounds)
__global__ __launch_bounds__(kScanThreads) void k_rebin_offsets(const int64_t* off, const int32_t* count, int64_t n,
                                                               int32_t headroom, int64_t* off_new) {
    __shared__ int64_t wsum[kScanThreads / 64];
    __shared__ int64_t carry;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) { carry = 0; off_new[0] = 0; }
    __syncthreads();
    for (int64_t base = 0; base < n; base += (int64_t)kScanThreads * kScanItems) {
        const int64_t c0 = base + (int64_t)t * kScanItems;
        int64_t v[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = c0 + k < n ? (int64_t)live_of(off, count, c0 + k) + headroom : 0;
        int64_t tot = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) { tot += v[k]; v[k] = tot; }
        // inclusive scan of the thread totals in the wavefront, then over the wavefronts
        int64_t inc = tot;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        int64_t before = carry;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        before += inc - tot;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (c0 + k < n) off_new[c0 + k + 1] = before + v[k];
        __syncthreads();
        if (t == 0) {
            int64_t r = 0;
            for (int w = 0; w < kScanThreads / 64; ++w) r += wsum[w];
            carry += r;
        }
        __syncthreads();
    }
}

// one wavefront per cell: the live records into the cell's new slab
__global__ __launch_bounds__(kThreads) void k_rebin_copy(Sp s, Sp d, int64_t n) {
    const int lane = threadIdx.x & 63;
    for (int64_t c = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); c < n;
         c += (int64_t)gridDim.x * (kThreads / 64)) {
        const int k = live_of(s.off, s.count, c);
        const int64_t a0 = s.off[c], b0 = d.off[c];
        for (int i = lane; i < k; i += 64) copy_rec(d, b0 + i, s, a0 + i);
        if (lane == 0) d.count[c] = k;
    }
}

Sp sp_of(const cmc_species* x) {
    return Sp{x->off, x->count, x->px, x->py, x->pz, x->w, x->parent};
}

unsigned mgrid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 3) / 4, 8192)); }

}  // namespace
}  // namespace cmc

using namespace cmc;

// the record arrays both sides carry: w always; the momenta on both or on neither
static cmc_status check_pair(const char* who, const cmc_species* d, const cmc_species* s) {
    CMC_REQUIRE(d && s && d->off && s->off && d->w && s->w, CMC_EINVAL, "%s: off and w are required", who);
    const bool dm = d->px && d->py && d->pz, sm = s->px && s->py && s->pz;
    CMC_REQUIRE(dm == sm && (dm || (!d->px && !d->py && !d->pz && !s->px && !s->py && !s->pz)), CMC_EINVAL,
                "%s: px, py, pz must be set on both species or on neither", who);
    for (const cmc_species* x : {d, s})
        CMC_REQUIRE(aligned_to<int64_t>(x->off) && aligned_to<int32_t>(x->count) && aligned_to<double>(x->px) &&
                        aligned_to<double>(x->py) && aligned_to<double>(x->pz) && aligned_to<double>(x->w) &&
                        aligned_to<int64_t>(x->parent),
                    CMC_EINVAL, "%s: an array is not aligned to its element type", who);
    return CMC_OK;
}

extern "C" cmc_status cmc_merge_species(int64_t n_cells, const cmc_species* dst, const cmc_species* src,
                                        int64_t* dropped, int32_t* status, void* stream) {
    const char* who = "cmc_merge_species";
    CMC_REQUIRE(n_cells >= 0, CMC_EINVAL, "%s: n_cells < 0", who);
    if (n_cells == 0) return CMC_OK;
    cmc_status s = check_pair(who, dst, src);
    if (s != CMC_OK) return s;
    CMC_REQUIRE(dst->count && src->count, CMC_EINVAL, "%s: both species need live counts", who);
    hipLaunchKernelGGL(k_merge, dim3(mgrid(n_cells)), dim3(kThreads), 0, as_stream(stream), sp_of(dst), sp_of(src),
                       n_cells, dropped, status);
    CMC_CHECK_LAUNCH(who);
    return CMC_OK;
}

extern "C" cmc_status cmc_rebin_offsets(int64_t n_cells, const cmc_species* src, int32_t headroom, int64_t* off_new,
                                        void* stream) {
    const char* who = "cmc_rebin_offsets";
    CMC_REQUIRE(n_cells >= 0, CMC_EINVAL, "%s: n_cells < 0", who);
    CMC_REQUIRE(headroom >= 0, CMC_EINVAL, "%s: headroom < 0", who);
    CMC_REQUIRE(src && src->off && off_new, CMC_EINVAL, "%s: NULL argument", who);
    CMC_REQUIRE(aligned_to<int64_t>(src->off) && aligned_to<int32_t>(src->count) && aligned_to<int64_t>(off_new),
                CMC_EINVAL, "%s: an array is not aligned to its element type", who);
    hipLaunchKernelGGL(k_rebin_offsets, dim3(1), dim3(kScanThreads), 0, as_stream(stream), src->off, src->count,
                       n_cells, headroom, off_new);
    CMC_CHECK_LAUNCH(who);
    return CMC_OK;
}

extern "C" cmc_status cmc_rebin_copy(int64_t n_cells, const cmc_species* src, const cmc_species* dst, void* stream) {
    const char* who = "cmc_rebin_copy";
    CMC_REQUIRE(n_cells >= 0, CMC_EINVAL, "%s: n_cells < 0", who);
    if (n_cells == 0) return CMC_OK;
    cmc_status s = check_pair(who, dst, src);
    if (s != CMC_OK) return s;
    CMC_REQUIRE(dst->count, CMC_EINVAL, "%s: the new species needs live counts", who);
    hipLaunchKernelGGL(k_rebin_copy, dim3(mgrid(n_cells)), dim3(kThreads), 0, as_stream(stream), sp_of(src),
                       sp_of(dst), n_cells);
    CMC_CHECK_LAUNCH(who);
    return CMC_OK;
}
