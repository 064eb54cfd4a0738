// dq_mixed.hip - streams with one block edge per 16^d super-block (gfx950).
//
// A workgroup owns a region of 4096 cells made of whole super-blocks: one
// 16^3 super-block in 3-D, a row of 16 super-blocks (16 x 256 cells) in 2-D,
// 256 super-blocks (4096 cells) in 1-D. Regions in row-major order are runs
// of super-blocks in stream order, so a region's blocks are a contiguous run
// of the pads and its outliers a contiguous run of the list.
//   encode: pre-quantisation into LDS (the codec's exact rounding), the
//           residual of every cell from its in-block lower neighbours in
//           LDS (zero halo; the origin takes q_o - P, the block's padding:
//           a constant halo cancels in every other Lorenzo difference,
//           Sections III-A and IV), codes to memory; a count pass, a scan
//           over regions, then an emit pass that walks the region in
//           stream order (block table in LDS) and writes its outliers;
//   decode: codes into LDS as residuals, the region's run of outliers
//           scattered onto the zero codes (checked: one outlier per zero
//           code, in stream order), then inclusive prefix sums along x, y,
//           z with a reset at every block start (the n-D inverse of the
//           Lorenzo residual), + P, dequantisation.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/dq_mixed.h"
#include "dq_host.hpp"

namespace dq {
namespace {

constexpr int kSuper = 16;
constexpr int kRegion = 4096;
constexpr int kMixThreads = 256;
constexpr int kPerThread = kRegion / kMixThreads;  // 16
constexpr int kMaxSb = 256;                       // super-blocks per region (1-D)
constexpr int kMaxBlocks = 1024;                  // blocks per region (1-D: 256 x 4)

// A dq_result as the kernels update it (status word first).
struct MixResult {
    int32_t status;
    uint32_t reserved;
    unsigned long long n_out;
    double eb_abs;
};

struct MixGeom {
    uint32_t d;
    uint32_t n[3];    // extents (z, y, x), 1 on absent axes
    uint32_t nsb[3];  // super-blocks per axis
    uint32_t R[3];    // region extents (z, y, x)
    uint32_t rsb;     // super-blocks per region along x
    uint32_t nrx;     // regions along x
    uint32_t n_regions;
    uint32_t n_super;
    uint64_t N;
};

bool make_mix_geom(const dq_params* p, MixGeom& g) {
    const int d = p->ndim;
    g.d = (uint32_t)d;
    g.N = 1;
    for (int a = 0; a < 3; ++a) {
        const int fa = a - (3 - d);
        g.n[a] = fa >= 0 ? (uint32_t)p->shape[fa] : 1u;
        g.nsb[a] = (g.n[a] + kSuper - 1) / kSuper;
        g.N *= g.n[a];
    }
    g.R[0] = d == 3 ? 16u : 1u;
    g.R[1] = d >= 2 ? 16u : 1u;
    g.R[2] = d == 3 ? 16u : (d == 2 ? 256u : 4096u);
    g.rsb = g.R[2] / kSuper;
    g.nrx = (g.nsb[2] + g.rsb - 1) / g.rsb;
    const uint64_t nr = (uint64_t)g.nsb[0] * g.nsb[1] * g.nrx;
    const uint64_t ns = (uint64_t)g.nsb[0] * g.nsb[1] * g.nsb[2];
    g.n_regions = (uint32_t)nr;
    g.n_super = (uint32_t)ns;
    return nr < 0x7fffffffull && ns < 0x7fffffffull;
}

__device__ __forceinline__ uint32_t edge_ok(uint8_t e, bool& bad) {
    if (e == 4 || e == 8 || e == 16) return e;
    bad = true;
    return 16u;
}

// Blocks of super-block s (edge E).
__device__ __forceinline__ uint32_t sb_blocks(const MixGeom& g, uint32_t s, uint32_t E) {
    const uint32_t sx = s % g.nsb[2], r = s / g.nsb[2];
    const uint32_t sy = r % g.nsb[1], sz = r / g.nsb[1];
    const uint32_t sc[3] = {sz, sy, sx};
    uint32_t nb = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool present = a >= 3 - (int)g.d;
        const uint32_t Ea = present ? E : 1u;
        const uint32_t ext = min((uint32_t)kSuper, g.n[a] - sc[a] * kSuper);
        nb *= present ? (ext + Ea - 1) / Ea : 1u;
    }
    return nb;
}

// One workgroup of 1024 threads: exclusive prefix of v(i), i < n, into out
// (n + 1 entries, out[n] = total); returns the total to every thread.
template <typename F>
__device__ uint32_t scan_all(uint32_t n, F v, uint32_t* out) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += 1024u) {
        const uint32_t i = base + (uint32_t)tid;
        const uint32_t x = i < n ? v(i) : 0u;
        const uint32_t incl = wave_scan_incl(x, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < 16; ++w) {
            before += w < wave ? wsum[w] : 0u;
            all += wsum[w];
        }
        const uint32_t carry = carry_s;
        if (i < n) out[i] = carry + before + incl - x;
        __syncthreads();
        if (tid == 0) carry_s = carry + all;
        __syncthreads();
    }
    const uint32_t total = carry_s;
    if (tid == 0) out[n] = total;
    return total;
}

__global__ __launch_bounds__(1024) void k_mixed_pad_off(MixGeom g, const uint8_t* __restrict__ edges,
                                                        uint32_t* __restrict__ pad_off, int32_t* status) {
    __shared__ int bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    scan_all(g.n_super, [&](uint32_t s) {
        bool bad = false;
        const uint32_t E = edge_ok(edges[s], bad);
        if (bad) bad_s = 1;
        return sb_blocks(g, s, E);
    }, pad_off);
    __syncthreads();
    if (threadIdx.x == 0 && bad_s && status) *status = DQ_EINVAL;
}

// Region state shared by the encode and the decode: the region's origin,
// its super-blocks' edges and pad offsets, and the block table in stream
// order (start of each block's cells in the region's stream order, its
// origin in region coordinates and its extents).
struct RegionLds {
    uint32_t pad_off[kMaxSb + 1];
    uint8_t edge[kMaxSb];
    uint32_t kstart[kMaxBlocks + 1];
    uint32_t korg[kMaxBlocks];  // lz << 24 | ly << 16 | lx (lx < 4096)
    uint32_t kext[kMaxBlocks];  // ez << 16 | ey << 8 | ex
    uint32_t n_sb, n_blk, cells;
    int bad;
};

struct RegionPos {
    uint32_t o[3];  // origin (z, y, x)
    uint32_t s0;    // first super-block
};

__device__ __forceinline__ RegionPos region_pos(const MixGeom& g, uint32_t r) {
    RegionPos p;
    const uint32_t rx = r % g.nrx, rr = r / g.nrx;
    const uint32_t ry = rr % g.nsb[1], rz = rr / g.nsb[1];
    p.o[0] = rz * g.R[0];
    p.o[1] = ry * g.R[1];
    p.o[2] = rx * g.R[2];
    p.s0 = (rz * g.nsb[1] + ry) * g.nsb[2] + rx * g.rsb;
    return p;
}

// Fills the block table of region r (all threads; ends with a barrier).
__device__ void region_table(const MixGeom& g, const RegionPos& rp, const uint8_t* __restrict__ edges,
                             const uint32_t* __restrict__ pad_off, RegionLds& L) {
    const int tid = threadIdx.x;
    const uint32_t n_sb = min(g.rsb, g.nsb[2] - rp.o[2] / kSuper);
    if (tid == 0) {
        L.n_sb = n_sb;
        L.bad = 0;
    }
    for (uint32_t i = tid; i <= n_sb; i += kMixThreads) L.pad_off[i] = pad_off[rp.s0 + i];
    for (uint32_t i = tid; i < n_sb; i += kMixThreads) {
        bool bad = false;
        L.edge[i] = (uint8_t)edge_ok(edges[rp.s0 + i], bad);
        if (bad) L.bad = 1;
    }
    __syncthreads();
    const uint32_t base = L.pad_off[0];
    const uint32_t n_blk = min(L.pad_off[n_sb] - base, (uint32_t)kMaxBlocks);
    // every thread describes up to 4 consecutive blocks
    uint32_t cnt[4];
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t k = (uint32_t)tid * 4u + (uint32_t)j;
        cnt[j] = 0;
        if (k >= n_blk) continue;
        // its super-block: the last i with pad_off[i] <= base + k
        uint32_t lo = 0, hi = n_sb;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (L.pad_off[mid] <= base + k) lo = mid;
            else hi = mid;
        }
        const uint32_t E = L.edge[lo];
        const uint32_t in_sb = base + k - L.pad_off[lo];
        const uint32_t sorg[3] = {rp.o[0], rp.o[1], rp.o[2] + lo * kSuper};  // super-block origin
        uint32_t nb[3], ext[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool present = a >= 3 - (int)g.d;
            const uint32_t Ea = present ? E : 1u;
            ext[a] = min((uint32_t)kSuper, g.n[a] - sorg[a]);
            if (!present) ext[a] = 1;
            nb[a] = (ext[a] + Ea - 1) / Ea;
        }
        const uint32_t bx = in_sb % nb[2], br = in_sb / nb[2];
        const uint32_t by = br % nb[1], bz = br / nb[1];
        const uint32_t bc[3] = {bz, by, bx};
        uint32_t org[3], e[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool present = a >= 3 - (int)g.d;
            const uint32_t Ea = present ? E : 1u;
            org[a] = sorg[a] + bc[a] * Ea - rp.o[a];
            e[a] = min(Ea, ext[a] - bc[a] * Ea);
        }
        L.korg[k] = (org[0] << 24) | (org[1] << 16) | org[2];
        L.kext[k] = (e[0] << 16) | (e[1] << 8) | e[2];
        cnt[j] = e[0] * e[1] * e[2];
        tot += cnt[j];
    }
    // exclusive scan of the block sizes in block order
    __shared__ uint32_t wsum[kMixThreads / 64];
    const int lane = tid & 63, wave = tid >> 6;
    const uint32_t incl = wave_scan_incl(tot, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kMixThreads / 64; ++w) {
        before += w < wave ? wsum[w] : 0u;
        all += wsum[w];
    }
    uint32_t run = before + incl - tot;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t k = (uint32_t)tid * 4u + (uint32_t)j;
        if (k < n_blk) L.kstart[k] = run;
        run += cnt[j];
    }
    if (tid == 0) {
        L.kstart[n_blk] = all;
        L.n_blk = n_blk;
        L.cells = all;
    }
    __syncthreads();
}

// Region-local cell c (z, y, x over R) -> its block's edge along each axis,
// whether it is the origin, and the block's index in the stream (global).
struct CellBlock {
    uint32_t E[3];
    uint32_t u[3];
    uint32_t gblk;
};

__device__ __forceinline__ CellBlock cell_block(const MixGeom& g, const RegionPos& rp, const RegionLds& L,
                                                const uint32_t (&l)[3]) {
    CellBlock cb;
    const uint32_t sbi = l[2] / kSuper;
    const uint32_t E = L.edge[sbi];
    const uint32_t sorg[3] = {rp.o[0], rp.o[1], rp.o[2] + sbi * kSuper};
    uint32_t nb[3], bc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool present = a >= 3 - (int)g.d;
        cb.E[a] = present ? E : 1u;
        const uint32_t ext = present ? min((uint32_t)kSuper, g.n[a] - sorg[a]) : 1u;
        nb[a] = (ext + cb.E[a] - 1) / cb.E[a];
        const uint32_t in_sb = rp.o[a] + l[a] - sorg[a];  // coordinate inside the super-block
        bc[a] = in_sb / cb.E[a];
        cb.u[a] = in_sb % cb.E[a];
    }
    cb.gblk = L.pad_off[sbi] + (bc[0] * nb[1] + bc[1]) * nb[2] + bc[2];
    return cb;
}

__device__ __forceinline__ void unflat(const MixGeom& g, uint32_t c, uint32_t (&l)[3]) {
    l[2] = c % g.R[2];
    const uint32_t r = c / g.R[2];
    l[1] = r % g.R[1];
    l[0] = r / g.R[1];
}

__device__ __forceinline__ bool cell_valid(const MixGeom& g, const RegionPos& rp, const uint32_t (&l)[3]) {
    return rp.o[0] + l[0] < g.n[0] && rp.o[1] + l[1] < g.n[1] && rp.o[2] + l[2] < g.n[2];
}

__device__ __forceinline__ uint64_t cell_index(const MixGeom& g, const RegionPos& rp, const uint32_t (&l)[3]) {
    return ((uint64_t)(rp.o[0] + l[0]) * g.n[1] + (rp.o[1] + l[1])) * g.n[2] + (rp.o[2] + l[2]);
}

__device__ __forceinline__ bool is_inlier_u(uint32_t u, uint32_t R) { return u - 1u < 2u * R - 1u; }

struct MixEncArgs {
    const float* x;
    const uint8_t* edges;
    const uint32_t* pad_off;
    const int32_t* pads;
    uint16_t* codes;
    uint32_t* out_idx;
    int32_t* out_val;
    uint64_t out_cap;
    uint32_t* region_cnt;  // n_regions + 1 (count pass), then exclusive offsets (scan)
    int32_t* status;
    const Scalars* sc;
    MixGeom g;
    uint32_t R;
};

// Pre-quantisation and residuals of region r into LDS (q, then delta).
__device__ void region_residuals(const MixEncArgs& a, const RegionPos& rp, RegionLds& L, uint32_t* dl) {
    const int tid = threadIdx.x;
    const double eb = a.sc->eb, twoeb = a.sc->twoeb, r = a.sc->r;
    uint64_t bad = 0;
    for (int j = 0; j < kPerThread; ++j) {  // uniform trip count: the exact path is wave-wide
        const uint32_t c = (uint32_t)tid + (uint32_t)j * kMixThreads;
        uint32_t l[3];
        unflat(a.g, c, l);
        const bool v = cell_valid(a.g, rp, l);
        float xv[1] = {v ? a.x[cell_index(a.g, rp, l)] : 0.0f};
        uint32_t q[1];
        prequant<1>(xv, r, twoeb, eb, q, bad);
        dl[c] = v ? q[0] : 0u;
    }
    if (bad && (tid & 63) == 0) __hip_atomic_store(a.status, (int)DQ_ERANGE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    uint32_t d[kPerThread];
    for (int j = 0; j < kPerThread; ++j) {
        const uint32_t c = (uint32_t)tid + (uint32_t)j * kMixThreads;
        uint32_t l[3];
        unflat(a.g, c, l);
        d[j] = 0;
        if (!cell_valid(a.g, rp, l)) continue;
        const CellBlock cb = cell_block(a.g, rp, L, l);
        if (cb.u[0] == 0 && cb.u[1] == 0 && cb.u[2] == 0) {  // the origin: q_o - P
            d[j] = dl[c] - (uint32_t)a.pads[cb.gblk];
            continue;
        }
        // sum over the lower corners S inside the block of (-1)^|S| q(c - 1_S)
        const uint32_t stride[3] = {a.g.R[1] * a.g.R[2], a.g.R[2], 1u};
        uint32_t acc = 0;
        for (int S = 0; S < 8; ++S) {
            bool in = true;
            uint32_t cc = c;
            int sign = 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                if (S & (1 << ax)) {
                    in = in && cb.u[ax] >= 1u;
                    cc -= stride[ax];
                    sign ^= 1;
                }
            }
            if (in) acc = sign ? acc - dl[cc] : acc + dl[cc];
        }
        d[j] = acc;
    }
    __syncthreads();
    for (int j = 0; j < kPerThread; ++j) dl[(uint32_t)tid + (uint32_t)j * kMixThreads] = d[j];
    __syncthreads();
}

// mode 0: codes and the region's outlier count; mode 1: the region's outliers
// (regions with none return at once).
template <int MODE>
__global__ __launch_bounds__(kMixThreads) void k_mixed_encode(MixEncArgs a) {
    __shared__ RegionLds L;
    __shared__ uint32_t dl[kRegion];
    __shared__ uint32_t wsum[kMixThreads / 64];
    const uint32_t r = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (MODE == 1) {
        if (a.region_cnt[r + 1] == a.region_cnt[r]) return;
        if (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != DQ_OK) return;
    }
    const RegionPos rp = region_pos(a.g, r);
    region_table(a.g, rp, a.edges, a.pad_off, L);
    region_residuals(a, rp, L, dl);
    const uint32_t R = a.R;
    if (MODE == 0) {
        uint32_t cnt = 0;
        for (int j = 0; j < kPerThread; ++j) {
            const uint32_t c = (uint32_t)tid + (uint32_t)j * kMixThreads;
            uint32_t l[3];
            unflat(a.g, c, l);
            if (!cell_valid(a.g, rp, l)) continue;
            const uint32_t u = dl[c] + R;
            const bool inl = is_inlier_u(u, R);
            a.codes[cell_index(a.g, rp, l)] = (uint16_t)(inl ? u : 0u);
            cnt += inl ? 0u : 1u;
        }
        const uint32_t incl = wave_scan_incl(cnt, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        if (tid == 0) {
            a.region_cnt[r] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
            if (L.bad) __hip_atomic_store(a.status, (int)DQ_EINVAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    // emit: thread t walks stream positions 16 t .. 16 t + 15 of the region
    uint32_t cnt = 0;
    uint32_t cell_of[kPerThread];
    for (int j = 0; j < kPerThread; ++j) {
        const uint32_t P = (uint32_t)tid * kPerThread + (uint32_t)j;
        cell_of[j] = 0xffffffffu;
        if (P >= L.cells) continue;
        uint32_t lo = 0, hi = L.n_blk;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (L.kstart[mid] <= P) lo = mid;
            else hi = mid;
        }
        const uint32_t off = P - L.kstart[lo];
        const uint32_t og = L.korg[lo], ex = L.kext[lo];
        const uint32_t e1 = (ex >> 8) & 0xffu, e2 = ex & 0xffu;
        const uint32_t lx = (og & 0xffffu) + off % e2;
        const uint32_t ly = ((og >> 16) & 0xffu) + (off / e2) % e1;
        const uint32_t lz = (og >> 24) + off / (e2 * e1);
        const uint32_t c = (lz * a.g.R[1] + ly) * a.g.R[2] + lx;
        if (!is_inlier_u(dl[c] + R, R)) {
            cell_of[j] = c;
            ++cnt;
        }
    }
    const uint32_t incl = wave_scan_incl(cnt, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    uint64_t pos = (uint64_t)a.region_cnt[r] + before + incl - cnt;
    for (int j = 0; j < kPerThread; ++j) {
        const uint32_t c = cell_of[j];
        if (c == 0xffffffffu) continue;
        uint32_t l[3];
        unflat(a.g, c, l);
        if (pos < a.out_cap) {
            a.out_idx[pos] = (uint32_t)cell_index(a.g, rp, l);
            a.out_val[pos] = (int32_t)dl[c];
        }
        ++pos;
    }
}

// Exclusive offsets of the regions' outlier counts, the call's outlier count
// and the capacity verdict.
__global__ __launch_bounds__(1024) void k_mixed_scan(uint32_t* region_cnt, uint32_t n_regions, MixResult* res,
                                                     uint64_t out_cap) {
    // in place: every count of a chunk is read before the chunk's offsets are written
    const uint32_t total = scan_all(n_regions, [&](uint32_t i) { return region_cnt[i]; }, region_cnt);
    if (threadIdx.x == 0 && __hip_atomic_load(&res->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == DQ_OK) {
        res->n_out = total;
        if (total > out_cap) __hip_atomic_store(&res->status, (int)DQ_ECAPACITY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (threadIdx.x == 0) {
        res->n_out = total;
    }
}

// ------------------------------------------------------------------ decode

struct MixDecArgs {
    const uint8_t* edges;
    const uint32_t* pad_off;
    const int32_t* pads;
    const uint16_t* codes;
    const uint32_t* out_idx;
    const int32_t* out_val;
    uint32_t n_out;
    float* x_hat;
    uint32_t* region_start;  // n_regions + 1
    MixResult* res;
    double twoeb;
    MixGeom g;
    uint32_t R;
};

__device__ __forceinline__ uint32_t region_of_index(const MixGeom& g, uint32_t idx) {
    if ((uint64_t)idx >= g.N) return g.n_regions;
    const uint32_t x = idx % g.n[2], r = idx / g.n[2];
    const uint32_t y = r % g.n[1], z = r / g.n[1];
    return ((z / g.R[0]) * g.nsb[1] + (g.d >= 2 ? y / g.R[1] : 0u)) * g.nrx + x / g.R[2];
}

// region_start[r] = first outlier of region r or later (r = 0..n_regions);
// also initialises the call's result.
__global__ __launch_bounds__(256) void k_mixed_index(MixDecArgs a, double eb_abs) {
    const uint32_t r = blockIdx.x * 256u + threadIdx.x;
    if (r == 0) {
        a.res->status = DQ_OK;
        a.res->reserved = 0;
        a.res->n_out = a.n_out;
        a.res->eb_abs = eb_abs;
    }
    if (r > a.g.n_regions) return;
    uint32_t lo = 0, hi = a.n_out;  // first entry whose region >= r
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (region_of_index(a.g, a.out_idx[mid]) < r) lo = mid + 1;
        else hi = mid;
    }
    a.region_start[r] = lo;
}

__global__ __launch_bounds__(kMixThreads) void k_mixed_decode(MixDecArgs a) {
    __shared__ RegionLds L;
    __shared__ uint32_t dl[kRegion];
    __shared__ uint32_t wsum[kMixThreads / 64];
    __shared__ int corrupt_s;
    const uint32_t r = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) corrupt_s = 0;
    const RegionPos rp = region_pos(a.g, r);
    region_table(a.g, rp, a.edges, a.pad_off, L);
    const uint32_t R = a.R;
    uint32_t zeros = 0;
    for (int j = 0; j < kPerThread; ++j) {
        const uint32_t c = (uint32_t)tid + (uint32_t)j * kMixThreads;
        uint32_t l[3];
        unflat(a.g, c, l);
        uint32_t v = 0;
        if (cell_valid(a.g, rp, l)) {
            const uint32_t code = a.codes[cell_index(a.g, rp, l)];
            v = code - R;
            zeros += code == 0 ? 1u : 0u;
        }
        dl[c] = v;
    }
    const uint32_t incl = wave_scan_incl(zeros, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    const uint32_t n_zero = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    const uint32_t e0 = a.region_start[r], e1 = a.region_start[r + 1];
    if (e1 < e0 || e1 - e0 != n_zero) corrupt_s = 1;
    // the run's entries: inside the region, on zero codes, in stream order
    if (e1 >= e0 && e1 - e0 == n_zero) {
        for (uint32_t e = e0 + (uint32_t)tid; e < e1; e += kMixThreads) {
            const uint32_t idx = a.out_idx[e];
            bool ok = region_of_index(a.g, idx) == r;
            uint32_t P = 0, c = 0;
            if (ok) {
                const uint32_t x = idx % a.g.n[2], rr = idx / a.g.n[2];
                const uint32_t y = rr % a.g.n[1], z = rr / a.g.n[1];
                const uint32_t l[3] = {z - rp.o[0], y - rp.o[1], x - rp.o[2]};
                c = (l[0] * a.g.R[1] + l[1]) * a.g.R[2] + l[2];
                const CellBlock cb = cell_block(a.g, rp, L, l);
                const uint32_t k = cb.gblk - L.pad_off[0];
                const uint32_t ex = L.kext[k];
                const uint32_t e1x = (ex >> 8) & 0xffu, e2x = ex & 0xffu;
                P = L.kstart[k] + (cb.u[0] * e1x + cb.u[1]) * e2x + cb.u[2];
                ok = a.codes[idx] == 0;
            }
            if (ok && e > e0) {  // strictly after the previous entry in stream order
                const uint32_t pidx = a.out_idx[e - 1];
                if (region_of_index(a.g, pidx) != r) {
                    ok = false;
                } else {
                    const uint32_t x = pidx % a.g.n[2], rr = pidx / a.g.n[2];
                    const uint32_t y = rr % a.g.n[1], z = rr / a.g.n[1];
                    const uint32_t l[3] = {z - rp.o[0], y - rp.o[1], x - rp.o[2]};
                    const CellBlock cb = cell_block(a.g, rp, L, l);
                    const uint32_t k = cb.gblk - L.pad_off[0];
                    const uint32_t ex = L.kext[k];
                    const uint32_t e1x = (ex >> 8) & 0xffu, e2x = ex & 0xffu;
                    const uint32_t Pp = L.kstart[k] + (cb.u[0] * e1x + cb.u[1]) * e2x + cb.u[2];
                    ok = Pp < P;
                }
            }
            if (ok) dl[c] = (uint32_t)a.out_val[e];
            else corrupt_s = 1;
        }
    }
    __syncthreads();
    // inclusive prefix sums inside the blocks: along x, then y, then z
    const uint32_t RZ = a.g.R[0], RY = a.g.R[1], RX = a.g.R[2];
    {
        const uint32_t t = (uint32_t)tid;  // segment (lz, ly, super-block column)
        const uint32_t nseg = RX / kSuper;
        const uint32_t sbi = t % nseg, rr = t / nseg;
        const uint32_t ly = rr % RY, lz = rr / RY;
        const uint32_t E = L.edge[min(sbi, L.n_sb - 1)];
        uint32_t s = 0;
        for (uint32_t i = 0; i < kSuper; ++i) {
            const uint32_t c = (lz * RY + ly) * RX + sbi * kSuper + i;
            s = (i % E == 0) ? dl[c] : s + dl[c];
            dl[c] = s;
        }
    }
    __syncthreads();
    if (a.g.d >= 2) {
        const uint32_t t = (uint32_t)tid;  // line (lz, lx) along y
        const uint32_t lx = t % RX, lz = t / RX;
        const uint32_t E = L.edge[min(lx / kSuper, L.n_sb - 1)];
        uint32_t s = 0;
        for (uint32_t i = 0; i < RY; ++i) {
            const uint32_t c = (lz * RY + i) * RX + lx;
            s = (i % E == 0) ? dl[c] : s + dl[c];
            dl[c] = s;
        }
        __syncthreads();
    }
    if (a.g.d == 3) {
        const uint32_t t = (uint32_t)tid;  // line (ly, lx) along z
        const uint32_t lx = t % RX, ly = t / RX;
        const uint32_t E = L.edge[0];
        uint32_t s = 0;
        for (uint32_t i = 0; i < RZ; ++i) {
            const uint32_t c = (i * RY + ly) * RX + lx;
            s = (i % E == 0) ? dl[c] : s + dl[c];
            dl[c] = s;
        }
        __syncthreads();
    }
    for (int j = 0; j < kPerThread; ++j) {
        const uint32_t c = (uint32_t)tid + (uint32_t)j * kMixThreads;
        uint32_t l[3];
        unflat(a.g, c, l);
        if (!cell_valid(a.g, rp, l)) continue;
        const CellBlock cb = cell_block(a.g, rp, L, l);
        const int32_t q = (int32_t)(dl[c] + (uint32_t)a.pads[cb.gblk]);
        a.x_hat[cell_index(a.g, rp, l)] = (float)((double)q * a.twoeb);
    }
    if (tid == 0 && (corrupt_s || L.bad))
        __hip_atomic_store(&a.res->status, corrupt_s ? (int)DQ_ECORRUPT : (int)DQ_EINVAL, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_mixed_init(Scalars* sc, MixResult* res, double eb) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc->eb = eb;
    sc->twoeb = 2.0 * eb;
    sc->r = 1.0 / (2.0 * eb);
    res->status = DQ_OK;
    res->reserved = 0;
    res->n_out = 0;
    res->eb_abs = eb;
}

dq_status mixed_check(const dq_params* p, MixGeom& g) {
    if (!p || p->ndim < 1 || p->ndim > 3) return DQ_EINVAL;
    double total = 1.0;
    for (int a = 0; a < p->ndim; ++a) {
        if (p->shape[a] < 1) return DQ_EINVAL;
        total *= (double)p->shape[a];
    }
    if (total > 4294967295.0) return DQ_EINVAL;
    if (p->radius < 1 || p->radius > 32768) return DQ_EINVAL;
    if (!make_mix_geom(p, g)) return DQ_EINVAL;
    return DQ_OK;
}

uint64_t mixed_ws_bytes(const MixGeom& g) {
    return host::align_up(sizeof(Scalars)) + host::align_up(4ull * ((uint64_t)g.n_regions + 1));
}

dq_status launched() { return hipGetLastError() == hipSuccess ? DQ_OK : DQ_EDEVICE; }

// ------------------------------------------------------------------ edge choice

constexpr uint8_t kEdges[3] = {4, 8, 16};

// Exhaustive edge of every super-block: the lowest cost of the three, ties to
// the larger edge.
__global__ void k_super_label(const unsigned long long* __restrict__ cost, uint32_t n_super,
                              uint8_t* __restrict__ edges, int32_t* __restrict__ label) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_super) return;
    int best = 2;
    for (int i = 1; i >= 0; --i)
        if (cost[(uint64_t)i * n_super + s] < cost[(uint64_t)best * n_super + s]) best = i;
    if (edges) edges[s] = kEdges[best];
    if (label) label[s] = best;
}

// The network's edge of every super-block: the block-size logits (outputs 5,
// 6, 7 of each sample) summed over the super-block's blocks at the base
// edge, the largest sum, ties to the larger edge. One thread per super-block.
__global__ void k_super_vote(MixGeom g, uint32_t base, const float* __restrict__ logits, uint8_t* __restrict__ edges,
                             int32_t* __restrict__ label) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n_super) return;
    const uint32_t sx = s % g.nsb[2], r = s / g.nsb[2];
    const uint32_t sy = r % g.nsb[1], sz = r / g.nsb[1];
    const uint32_t sc[3] = {sz, sy, sx};
    uint32_t nb[3], lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool present = a >= 3 - (int)g.d;
        const uint32_t Ea = present ? base : 1u;
        nb[a] = (g.n[a] + Ea - 1) / Ea;  // blocks per axis of the field at the base edge
        lo[a] = present ? sc[a] * (kSuper / base) : 0u;
        hi[a] = present ? min(nb[a], lo[a] + kSuper / base) : 1u;
    }
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (uint32_t bz = lo[0]; bz < hi[0]; ++bz)
        for (uint32_t by = lo[1]; by < hi[1]; ++by)
            for (uint32_t bx = lo[2]; bx < hi[2]; ++bx) {
                const uint64_t b = ((uint64_t)bz * nb[1] + by) * nb[2] + bx;
#pragma unroll
                for (int i = 0; i < 3; ++i) acc[i] += logits[b * 8 + 5 + i];
            }
    int best = 2;
    for (int i = 1; i >= 0; --i)
        if (acc[i] > acc[best]) best = i;
    if (edges) edges[s] = kEdges[best];
    if (label) label[s] = best;
}

// Pads of a mixed stream from per-edge pads in uniform block order: block b
// of super-block s (edge E) takes pads_E at its uniform block index. One
// workgroup per super-block, a thread per block.
__global__ __launch_bounds__(64) void k_mixed_gather(MixGeom g, const uint8_t* __restrict__ edges,
                                                     const uint32_t* __restrict__ pad_off,
                                                     const int32_t* __restrict__ p4, const int32_t* __restrict__ p8,
                                                     const int32_t* __restrict__ p16, int32_t* __restrict__ pads) {
    const uint32_t s = blockIdx.x;
    bool bad = false;
    const uint32_t E = edge_ok(edges[s], bad);
    const int32_t* src = E == 4 ? p4 : (E == 8 ? p8 : p16);
    const uint32_t sx = s % g.nsb[2], r = s / g.nsb[2];
    const uint32_t sy = r % g.nsb[1], sz = r / g.nsb[1];
    const uint32_t sc[3] = {sz, sy, sx};
    uint32_t nbf[3], nbs[3], org[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool present = a >= 3 - (int)g.d;
        const uint32_t Ea = present ? E : 1u;
        nbf[a] = (g.n[a] + Ea - 1) / Ea;  // field's blocks per axis at this edge
        const uint32_t ext = present ? min((uint32_t)kSuper, g.n[a] - sc[a] * kSuper) : 1u;
        nbs[a] = (ext + Ea - 1) / Ea;     // the super-block's
        org[a] = present ? sc[a] * (kSuper / Ea) : 0u;
    }
    const uint32_t n = nbs[0] * nbs[1] * nbs[2];
    for (uint32_t k = threadIdx.x; k < n; k += 64) {
        const uint32_t bx = k % nbs[2], kr = k / nbs[2];
        const uint32_t by = kr % nbs[1], bz = kr / nbs[1];
        const uint64_t u = ((uint64_t)(org[0] + bz) * nbf[1] + (org[1] + by)) * nbf[2] + (org[2] + bx);
        pads[pad_off[s] + k] = src[u];
    }
}

}  // namespace
}  // namespace dq

using namespace dq;

extern "C" {

dq_status dq_mixed_num_super(const dq_params* p, uint64_t* n_super) {
    MixGeom g;
    const dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (!n_super) return DQ_EINVAL;
    *n_super = g.n_super;
    return DQ_OK;
}

dq_status dq_mixed_pad_offsets(const dq_params* p, const uint8_t* edges, uint32_t* pad_off, int32_t* status,
                               void* hip_stream) {
    MixGeom g;
    const dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (!edges || !pad_off) return DQ_EINVAL;
    hipLaunchKernelGGL(k_mixed_pad_off, dim3(1), dim3(1024), 0, reinterpret_cast<hipStream_t>(hip_stream), g, edges,
                       pad_off, status);
    return launched();
}

dq_status dq_mixed_workspace(const dq_params* p, uint64_t* bytes) {
    MixGeom g;
    const dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (!bytes) return DQ_EINVAL;
    *bytes = mixed_ws_bytes(g);
    return DQ_OK;
}

dq_status dq_mixed_compress(const dq_params* p, const float* x, const uint8_t* edges, const uint32_t* pad_off,
                            const int32_t* pads, uint16_t* codes, uint32_t* out_idx, int32_t* out_val,
                            uint64_t out_cap, dq_result* res, void* ws, uint64_t ws_bytes, void* hip_stream) {
    MixGeom g;
    dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (p->eb_mode != DQ_EB_ABS || !(p->eb > 0.0) || !std::isfinite(p->eb) || !std::isfinite(1.0 / (2.0 * p->eb)))
        return DQ_EINVAL;
    if (!x || !edges || !pad_off || !pads || !codes || !res || !ws) return DQ_EINVAL;
    if (out_cap > 0 && (!out_idx || !out_val)) return DQ_EINVAL;
    if ((reinterpret_cast<uintptr_t>(res) % 8) || (reinterpret_cast<uintptr_t>(ws) % host::kAlign)) return DQ_EINVAL;
    if (ws_bytes < mixed_ws_bytes(g)) return DQ_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* w = static_cast<char*>(ws);
    Scalars* sc = reinterpret_cast<Scalars*>(w);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(w + host::align_up(sizeof(Scalars)));
    MixResult* rv = reinterpret_cast<MixResult*>(res);
    hipLaunchKernelGGL(k_mixed_init, dim3(1), dim3(64), 0, s, sc, rv, p->eb);
    MixEncArgs a;
    a.x = x;
    a.edges = edges;
    a.pad_off = pad_off;
    a.pads = pads;
    a.codes = codes;
    a.out_idx = out_idx;
    a.out_val = out_val;
    a.out_cap = out_cap;
    a.region_cnt = cnt;
    a.status = &res->status;
    a.sc = sc;
    a.g = g;
    a.R = (uint32_t)p->radius;
    hipLaunchKernelGGL(k_mixed_encode<0>, dim3(g.n_regions), dim3(kMixThreads), 0, s, a);
    hipLaunchKernelGGL(k_mixed_scan, dim3(1), dim3(1024), 0, s, cnt, g.n_regions, rv, out_cap);
    hipLaunchKernelGGL(k_mixed_encode<1>, dim3(g.n_regions), dim3(kMixThreads), 0, s, a);
    return launched();
}

dq_status dq_mixed_decompress(const dq_params* p, double eb_abs, const uint8_t* edges, const uint32_t* pad_off,
                              const int32_t* pads, const uint16_t* codes, const uint32_t* out_idx,
                              const int32_t* out_val, uint64_t n_out, float* x_hat, dq_result* res, void* ws,
                              uint64_t ws_bytes, void* hip_stream) {
    MixGeom g;
    dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (!(eb_abs > 0.0) || !std::isfinite(eb_abs)) return DQ_EINVAL;
    if (!edges || !pad_off || !pads || !codes || !x_hat || !res || !ws) return DQ_EINVAL;
    if (n_out > 0 && (!out_idx || !out_val)) return DQ_EINVAL;
    if (n_out > g.N) return DQ_EINVAL;
    if ((reinterpret_cast<uintptr_t>(res) % 8) || (reinterpret_cast<uintptr_t>(ws) % host::kAlign)) return DQ_EINVAL;
    if (ws_bytes < mixed_ws_bytes(g)) return DQ_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* w = static_cast<char*>(ws);
    MixDecArgs a;
    a.edges = edges;
    a.pad_off = pad_off;
    a.pads = pads;
    a.codes = codes;
    a.out_idx = out_idx;
    a.out_val = out_val;
    a.n_out = (uint32_t)n_out;
    a.x_hat = x_hat;
    a.region_start = reinterpret_cast<uint32_t*>(w + host::align_up(sizeof(Scalars)));
    a.res = reinterpret_cast<MixResult*>(res);
    a.twoeb = 2.0 * eb_abs;
    a.g = g;
    a.R = (uint32_t)p->radius;
    hipLaunchKernelGGL(k_mixed_index, dim3((g.n_regions + 1 + 255) / 256), dim3(256), 0, s, a, eb_abs);
    hipLaunchKernelGGL(k_mixed_decode, dim3(g.n_regions), dim3(kMixThreads), 0, s, a);
    return launched();
}

dq_status dq_super_label(const dq_params* p, const uint64_t* cost, uint8_t* edges, int32_t* label,
                         void* hip_stream) {
    MixGeom g;
    const dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (!cost || (!edges && !label)) return DQ_EINVAL;
    hipLaunchKernelGGL(k_super_label, dim3((g.n_super + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), reinterpret_cast<const unsigned long long*>(cost),
                       g.n_super, edges, label);
    return launched();
}

dq_status dq_super_vote(const dq_params* p, int32_t base, const float* logits, uint8_t* edges, int32_t* label,
                        void* hip_stream) {
    MixGeom g;
    const dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (base != 4 && base != 8 && base != 16) return DQ_EINVAL;
    if (!logits || (!edges && !label)) return DQ_EINVAL;
    hipLaunchKernelGGL(k_super_vote, dim3((g.n_super + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), g, (uint32_t)base, logits, edges, label);
    return launched();
}

dq_status dq_mixed_gather_pads(const dq_params* p, const uint8_t* edges, const uint32_t* pad_off,
                               const int32_t* pads4, const int32_t* pads8, const int32_t* pads16, int32_t* pads,
                               void* hip_stream) {
    MixGeom g;
    const dq_status st = mixed_check(p, g);
    if (st != DQ_OK) return st;
    if (!edges || !pad_off || !pads4 || !pads8 || !pads16 || !pads) return DQ_EINVAL;
    hipLaunchKernelGGL(k_mixed_gather, dim3(g.n_super), dim3(64), 0, reinterpret_cast<hipStream_t>(hip_stream), g,
                       edges, pad_off, pads4, pads8, pads16, pads);
    return launched();
}

}  // extern "C"
