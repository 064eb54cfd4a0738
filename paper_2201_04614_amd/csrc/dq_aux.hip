// dq_aux.hip - small kernels around the encode/decode passes (gfx950).
//
//  compress:   [ABS] init | [REL] min/max pass (which initialises the call;
//              the consuming kernels resolve the bound per workgroup) ->
//              [GLOBAL] sum of q -> encode -> scan of per-tile outlier counts and scatter
//              of the staged outliers into block-major order (one fused
//              kernel up to kPlaceTiles tiles, three kernels beyond)
//  decompress: [n_out > 0] per-block start of the outlier list (and
//              validation of its order) -> decode (which also initialises the
//              call's result)
// Status words are written with plain stores of one error value; the only
// device errors of a compress call are EINVAL/ERANGE (before or during encode)
// and ECAPACITY (decided by the scan when no other error occurred); decode
// only reports ECORRUPT.
#include "dq_device.hpp"
#include "dq_fastdiv.hpp"
#include "dq_kernels.hpp"

namespace dq {

struct ResultDev {
    int32_t status;
    uint32_t reserved;
    unsigned long long n_out;
    double eb_abs;
};

__device__ __forceinline__ void store_status(int32_t* status, int v) {
    __hip_atomic_store(status, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int load_status(const int32_t* status) {
    return __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ compress init

__device__ __forceinline__ void init_scalars(Scalars* sc, ResultDev* res) {
    sc->stage_count = 0;
    sc->sumq = 0;
    sc->gpad = 0;
    res->status = ST_OK;
    res->reserved = 0;
    res->n_out = 0;
}

// absolute bound given by the caller
__device__ __forceinline__ void compress_init(Scalars* sc, ResultDev* res, double eb) {
    init_scalars(sc, res);
    sc->eb = eb;
    sc->twoeb = 2.0 * eb;
    sc->r = 1.0 / (2.0 * eb);
    res->eb_abs = eb;
}

__global__ void k_compress_init(Scalars* sc, ResultDev* res, double eb) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    compress_init(sc, res, eb);
}

void launch_compress_init(Scalars* sc, void* res, double eb, hipStream_t stream) {
    hipLaunchKernelGGL(k_compress_init, dim3(1), dim3(64), 0, stream, sc, (ResultDev*)res, eb);
}

// ------------------------------------------------------------------ value range (REL bound)

// Running min / max of the values and a non-finite detector: fma(x, 0, acc)
// turns NaN for an infinite or NaN x and stays NaN. On finite data the float
// min / max are exact, so the bound equals the one over order-preserving
// keys; with any non-finite value the call fails with ERANGE anyway.
__device__ __forceinline__ void minmax_acc(float e, float& mn, float& mx, float& nfa) {
    mn = __builtin_fminf(mn, e);
    mx = __builtin_fmaxf(mx, e);
    nfa = __builtin_fmaf(e, 0.0f, nfa);
}

__device__ __forceinline__ void minmax_acc4(const f32x4 v, float& mn, float& mx, float& nfa) {
    mn = __builtin_fminf(mn, __builtin_fminf(__builtin_fminf(v.x, v.y), __builtin_fminf(v.z, v.w)));
    mx = __builtin_fmaxf(mx, __builtin_fmaxf(__builtin_fmaxf(v.x, v.y), __builtin_fmaxf(v.z, v.w)));
    nfa = __builtin_fmaf(v.x, 0.0f, nfa);
    nfa = __builtin_fmaf(v.y, 0.0f, nfa);
    nfa = __builtin_fmaf(v.z, 0.0f, nfa);
    nfa = __builtin_fmaf(v.w, 0.0f, nfa);
}

// Per-workgroup min / max keys and a non-finite flag (no atomics: every
// wave of the kernels that need the bound combines the partials, see
// bound_finish). First kernel of a compress call with a relative bound, so
// it also initialises the call.
__device__ __forceinline__ void minmax_part(const float* __restrict__ x, uint64_t N, uint2* parts, int vec4,
                                            Scalars* sc, ResultDev* res, uint32_t part, uint32_t nparts) {
    constexpr int W = kMinmaxThreads / 64;
    __shared__ float smin[W], smax[W], snf[W];
    if (part == 0 && threadIdx.x == 0) {
        init_scalars(sc, res);
        res->eb_abs = 0.0;
    }
    float mn = __builtin_inff(), mx = -__builtin_inff(), nfa = 0.0f;
    const uint64_t tid = (uint64_t)part * kMinmaxThreads + threadIdx.x;
    const uint64_t stride = (uint64_t)nparts * kMinmaxThreads;
    uint64_t start = 0;
    if (vec4) {
        const uint64_t n4 = N / 4;
        const f32x4* x4 = reinterpret_cast<const f32x4*>(x);
        uint64_t i = tid;
        for (; i + stride < n4; i += 2 * stride) {  // two 16-byte loads in flight
            const f32x4 v0 = x4[i];
            const f32x4 v1 = x4[i + stride];
            minmax_acc4(v0, mn, mx, nfa);
            minmax_acc4(v1, mn, mx, nfa);
        }
        for (; i < n4; i += stride) minmax_acc4(x4[i], mn, mx, nfa);
        start = n4 * 4;
    }
    for (uint64_t i = start + tid; i < N; i += stride) minmax_acc(x[i], mn, mx, nfa);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        mn = __builtin_fminf(mn, __shfl_xor(mn, off));
        mx = __builtin_fmaxf(mx, __shfl_xor(mx, off));
        nfa += __shfl_xor(nfa, off);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin[wave] = mn;
        smax[wave] = mx;
        snf[wave] = nfa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < W; ++w) {
            mn = __builtin_fminf(mn, smin[w]);
            mx = __builtin_fmaxf(mx, smax[w]);
            nfa += snf[w];
        }
        parts[part] = make_uint2(fkey(mn), nfa != nfa ? 0xffffffffu : fkey(mx));
    }
}

__global__ __launch_bounds__(kMinmaxThreads) void k_minmax(const float* __restrict__ x, uint64_t N, uint2* parts,
                                                           int vec4, Scalars* sc, ResultDev* res) {
    minmax_part(x, N, parts, vec4, sc, res, blockIdx.x, gridDim.x);
}

int launch_minmax(const AuxArgs& a, uint2* parts, void* res, hipStream_t stream) {
    const int vec4 = ((reinterpret_cast<uintptr_t>(a.x) & 15u) == 0) ? 1 : 0;
    uint64_t work = vec4 ? a.N / 4 : a.N;
    uint64_t blocks = (work + 4 * kMinmaxThreads - 1) / (4 * kMinmaxThreads);
    if (blocks > kMinmaxParts) blocks = kMinmaxParts;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_minmax, dim3((uint32_t)blocks), dim3(kMinmaxThreads), 0, stream, a.x, a.N, parts, vec4,
                       a.sc, (ResultDev*)res);
    return (int)blocks;
}

// ------------------------------------------------------------------ global mean of q

__global__ __launch_bounds__(256) void k_sumq(const float* __restrict__ x, uint64_t N, Scalars* sc,
                                              int32_t* status, BoundArgs bound) {
    __shared__ long long ssum[4];
    __shared__ int sbad[4];
    uint4 pp[kBoundLoads];
    bound_fetch(bound, pp, threadIdx.x & 63);
    const Bound bd = bound_finish(bound, pp, threadIdx.x & 63);  // an invalid bound is reported by encode
    if (bd.status != ST_OK || load_status(status) != ST_OK) return;
    const double r = bd.r, twoeb = bd.twoeb, eb = bd.eb;
    long long s = 0;
    uint64_t bad = 0;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // uniform trip count so the wave-wide near-half check in prequant sees all lanes
    const uint64_t iters = (N + stride - 1) / stride;
    for (uint64_t it = 0; it < iters; ++it) {
        const uint64_t i = tid + it * stride;
        float v[1] = {i < N ? x[i] : 0.0f};
        uint32_t q[1];
        prequant<1>(v, r, twoeb, eb, q, bad);
        s += (int32_t)q[0];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    const bool anybad = bad != 0;
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ssum[wave] = s;
        sbad[wave] = anybad ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = ssum[0] + ssum[1] + ssum[2] + ssum[3];
        atomicAdd(&sc->sumq, (unsigned long long)t);  // one atomic per workgroup
        if (sbad[0] | sbad[1] | sbad[2] | sbad[3]) store_status(status, ST_ERANGE);
    }
}

void launch_sumq(const AuxArgs& a, const BoundArgs& bound, hipStream_t stream) {
    uint64_t blocks = (a.N + 1023) / 1024;
    if (blocks > 512) blocks = 512;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_sumq, dim3((uint32_t)blocks), dim3(256), 0, stream, a.x, a.N, a.sc, a.status, bound);
}

// ------------------------------------------------------------------ large fields: chunked scan + scatter

// Fields of more than kPlaceTiles tiles take three kernels. The tiles are cut
// into chunks of kChunkTiles; k_chunk_sums writes each chunk's outlier total;
// k_scatter_chunks (kChunkSplit workgroups per chunk, since outliers cluster
// in a few chunks of fields with sharp features) turns them into the chunk's
// carry, scans its tile counts into tile_off and places the entries of its
// tiles' staging regions; k_scatter_overflow places the overflow list, whose
// entries may belong to any tile.

// Dense staging: a wave copies tile t's outliers (tile offset toff, `total`
// of them) from their slots to the list, 64 blocks at a time: lane j reads
// block j's in-tile prefix, a wave scan gives each block's run, and the
// lanes then take consecutive list entries (four loads in flight each),
// finding the block of an entry by a search over the lanes' prefixes. The
// list positions are consecutive, so the stores coalesce. Positions at or
// past n are not written.
__device__ __forceinline__ void place_tile_dense(const Staging& stg, const Geom& g, uint32_t t, uint32_t toff,
                                                 uint32_t total, const uint32_t* __restrict__ block_info,
                                                 uint32_t n, uint32_t* __restrict__ out_idx,
                                                 int32_t* __restrict__ out_val, int lane) {
    const uint32_t tx = t % g.ntx;
    const uint32_t bx0 = tx * g.bpt;
    const uint32_t nb = min(g.bpt, g.nbx - bx0);
    const uint32_t blk0 = (t / g.ntx) * g.nbx + bx0;
    const uint2* reg = reinterpret_cast<const uint2*>(stg.region + (uint64_t)t * stg.spt);
    for (uint32_t j0 = 0; j0 < nb; j0 += 64) {
        const uint32_t j = j0 + (uint32_t)lane;
        const bool in = j < nb;
        const uint32_t info = in ? block_info[blk0 + j] : 0u;
        const uint32_t nxt = (j + 1 < nb) ? (block_info[blk0 + j + 1] & ~kOriginFlag) : total;
        const uint32_t cur = info & ~kOriginFlag;
        const uint32_t cnt = in ? min(nxt - cur, stg.bcells) : 0u;  // at most the block's cells
        const uint32_t skip = (info & kOriginFlag) ? 0u : 1u;
        const uint32_t incl = wave_scan_incl(cnt, lane);
        const uint32_t excl = incl - cnt;               // lanes past nb: the chunk's total
        const uint32_t E = readlane(incl, 63);
        const uint32_t base = toff + readlane(cur, 0);  // list position of the chunk's first entry
        for (uint32_t k0 = 0; k0 < E; k0 += 256) {
            uint2 e[4];
            bool ok[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t q = k0 + (uint32_t)u * 64u + (uint32_t)lane;
                ok[u] = q < E;
                // the last lane (block) whose exclusive prefix is <= q
                int l = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1) {
                    const uint32_t v = (uint32_t)__shfl((int)excl, l + step);
                    if (v <= q) l += step;
                }
                const uint32_t r = q - (uint32_t)__shfl((int)excl, l);
                const uint32_t sk = (uint32_t)__shfl((int)skip, l);
                e[u] = ok[u] ? reg[(uint64_t)(j0 + (uint32_t)l) * stg.bcells + sk + r] : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t pos = base + k0 + (uint32_t)u * 64u + (uint32_t)lane;
                if (ok[u] && pos < n) {
                    out_idx[pos] = e[u].x;
                    out_val[pos] = (int32_t)e[u].y;
                }
            }
        }
    }
}

__device__ __forceinline__ uint32_t block_sum256(uint32_t v, uint32_t* red, int lane, int wave) {
    const uint32_t incl = wave_scan_incl(v, lane);
    if (lane == 63) red[wave] = incl;
    __syncthreads();
    const uint32_t t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void chunk_sum_part(const uint32_t* __restrict__ cnt, uint32_t n_tiles,
                                               uint32_t* __restrict__ chunk_sum, uint32_t chunk) {
    __shared__ uint32_t red[4];
    const int tid = threadIdx.x;
    const uint32_t t = chunk * kChunkTiles + (uint32_t)tid;
    const uint32_t v = t < n_tiles ? cnt[t] : 0u;
    const uint32_t s = block_sum256(v, red, tid & 63, tid >> 6);
    if (tid == 0) chunk_sum[chunk] = s;
}

__global__ __launch_bounds__(256) void k_chunk_sums(const uint32_t* __restrict__ cnt, uint32_t n_tiles,
                                                    uint32_t* __restrict__ chunk_sum) {
    chunk_sum_part(cnt, n_tiles, chunk_sum, blockIdx.x);
}

// Share `part` (of kChunkSplit) of chunk c's placement; the share (0, 0)
// writes the call's outlier count and capacity verdict.
__device__ __forceinline__ void scatter_chunk_part(const Staging& stg, ResultDev* res, uint64_t out_cap,
                                                   const uint32_t* __restrict__ cnt, uint32_t* __restrict__ tile_off,
                                                   const uint32_t* __restrict__ chunk_sum, uint32_t n_tiles,
                                                   uint32_t n_chunks, const uint32_t* __restrict__ block_info,
                                                   const Geom& g, uint32_t* __restrict__ out_idx,
                                                   int32_t* __restrict__ out_val, const uint32_t c,
                                                   const uint32_t part) {
    __shared__ uint32_t red[4], red2[4];
    __shared__ uint32_t eoff[kChunkTiles + 1];  // exclusive prefix of the region entries per tile
    __shared__ uint32_t toff_s[kChunkTiles];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // carry of this chunk and the field's total
    uint32_t before = 0, all = 0;
    for (uint32_t i = (uint32_t)tid; i < n_chunks; i += 256u) {
        const uint32_t v = chunk_sum[i];
        all += v;
        before += i < c ? v : 0u;
    }
    const uint32_t carry = block_sum256(before, red, lane, wave);
    const uint32_t total = block_sum256(all, red, lane, wave);
    // tile offsets, and the prefix of the entries held in the regions
    const uint32_t t = c * kChunkTiles + (uint32_t)tid;
    const uint32_t k = t < n_tiles ? cnt[t] : 0u;
    const uint32_t kr = min(k, stg.spt);
    const uint32_t inc = wave_scan_incl(k, lane);
    const uint32_t incr = wave_scan_incl(kr, lane);
    if (lane == 63) {
        red[wave] = inc;
        red2[wave] = incr;
    }
    __syncthreads();
    uint32_t wb = 0, wbr = 0;
    for (int w = 0; w < wave; ++w) {
        wb += red[w];
        wbr += red2[w];
    }
    const uint32_t off = carry + wb + inc - k;
    if (part == 0 && t < n_tiles) tile_off[t] = off;
    toff_s[tid] = off;
    eoff[tid + 1] = wbr + incr;
    if (tid == 0) eoff[0] = 0u;
    if (c == 0 && part == 0 && tid == 0 && load_status(&res->status) == ST_OK) {
        res->n_out = total;
        if (total > out_cap) store_status(&res->status, ST_ECAPACITY);
    }
    __syncthreads();
    if (total == 0 || total > out_cap || load_status(&res->status) != ST_OK) return;  // nothing, or incomplete
    if (stg.dense) {  // a wave per tile, the kChunkSplit workgroups of the chunk in turn
        for (uint32_t i = part * 4u + (uint32_t)wave; i < kChunkTiles; i += kChunkSplit * 4u) {
            const uint32_t tt = c * kChunkTiles + i;
            if (tt >= n_tiles) break;
            const uint32_t k = cnt[tt];
            if (k) place_tile_dense(stg, g, tt, toff_s[i], k, block_info, total, out_idx, out_val, lane);
        }
        return;
    }
    const uint32_t E = eoff[kChunkTiles];
    const uint64_t rbase = (uint64_t)c * kChunkTiles * stg.spt;
    // flattened walk over the chunk's region entries, four per thread at a
    // time; the kChunkSplit workgroups of a chunk take turns in strides of 1024
    for (uint32_t k0 = part * 1024u; k0 < E; k0 += kChunkSplit * 1024u) {
        uint4 e[4];
        uint32_t o[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t q = k0 + (uint32_t)u * 256u + (uint32_t)tid;
            ok[u] = q < E;
            // last tile j with eoff[j] <= q
            uint32_t lo = 0, hi = kChunkTiles;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (eoff[mid] <= q) lo = mid;
                else hi = mid;
            }
            o[u] = toff_s[lo];
            const uint64_t slot = rbase + (uint64_t)lo * stg.spt + (q - eoff[lo]);
            e[u] = ok[u] ? stg.region[slot] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (ok[u]) place_entry(e[u], o[u], block_info, total, out_idx, out_val);
    }
}

__global__ __launch_bounds__(256) void k_scatter_chunks(Staging stg, ResultDev* res, uint64_t out_cap,
                                                        const uint32_t* __restrict__ cnt,
                                                        uint32_t* __restrict__ tile_off,
                                                        const uint32_t* __restrict__ chunk_sum, uint32_t n_tiles,
                                                        uint32_t n_chunks, const uint32_t* __restrict__ block_info,
                                                        Geom g, uint32_t* __restrict__ out_idx,
                                                        int32_t* __restrict__ out_val) {
    scatter_chunk_part(stg, res, out_cap, cnt, tile_off, chunk_sum, n_tiles, n_chunks, block_info, g, out_idx,
                       out_val, blockIdx.x / kChunkSplit, blockIdx.x % kChunkSplit);
}

// ------------------------------------------------------------------ batches: one launch per stage

// Value-range pass (or the initialisation of a call with an absolute bound)
// of every field of a batch: workgroup k runs unit k = (field, part). Unit 0
// also clears the batch's tickets, and part 0 of a field clears its
// decompress status word (the decompress of a replayed graph then reports
// its own outcome).
__global__ __launch_bounds__(kMinmaxThreads) void k_batch_aux(const AuxField* __restrict__ fields,
                                                              const uint2* __restrict__ units,
                                                              unsigned int* tickets, uint32_t n_tickets) {
    const uint2 un = units[blockIdx.x];
    const AuxField f = fields[un.x];
    ResultDev* res = reinterpret_cast<ResultDev*>(f.res_);
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < n_tickets; i += blockDim.x) tickets[i] = 0u;
    if (un.y == 0 && threadIdx.x == 0) *f.dres_word = 0ull;
    if (f.nparts == 0) {
        if (threadIdx.x == 0) compress_init(f.sc, res, f.eb);
        return;
    }
    minmax_part(f.x, f.N, f.parts, f.vec4, f.sc, res, un.y, (uint32_t)f.nparts);
}

// The value range of every field with a value-range pass reduced to one
// (min key, max key) pair, so that each wave of the batch encode loads 16
// bytes instead of every partial: one wave per field.
__global__ __launch_bounds__(64) void k_batch_range(const AuxField* __restrict__ fields, uint2* __restrict__ reduced) {
    const AuxField f = fields[blockIdx.x];
    if (f.nparts == 0) return;
    const int lane = threadIdx.x;
    uint32_t kmin = 0xffffffffu, kmax = 0u;
    for (int i = lane; i < f.nparts; i += 64) {
        const uint2 v = f.parts[i];
        kmin = min(kmin, v.x);
        kmax = max(kmax, v.y);
    }
    kmin = wave_min_u32(kmin);
    kmax = wave_max_u32(kmax);
    if (lane == 0) reduced[2 * blockIdx.x] = make_uint2(kmin, kmax);
}

// Outlier totals of every 256-tile chunk of every field: unit = (field, chunk).
__global__ __launch_bounds__(256) void k_batch_chunk_sums(const PlaceField* __restrict__ fields,
                                                          const uint2* __restrict__ units) {
    const uint2 un = units[blockIdx.x];
    const PlaceField& f = fields[un.x];
    chunk_sum_part(f.cnt, f.n_tiles, f.chunk_sum, un.y);
}

// Tile offsets and outlier placement of every chunk of every field: unit =
// (field, chunk), kChunkSplit workgroups each.
__global__ __launch_bounds__(256) void k_batch_scatter(const PlaceField* __restrict__ fields,
                                                       const uint2* __restrict__ units) {
    const uint2 un = units[blockIdx.x / kChunkSplit];
    const PlaceField f = fields[un.x];
    scatter_chunk_part(f.stg, reinterpret_cast<ResultDev*>(f.res_), f.out_cap, f.cnt, f.tile_off, f.chunk_sum, f.n_tiles, f.n_chunks, f.block_info,
                       f.g, f.out_idx, f.out_val, un.y, blockIdx.x % kChunkSplit);
}

void launch_batch_aux(const AuxField* fields, uint32_t n_fields, const uint2* units, uint32_t n_units,
                      unsigned int* tickets, uint32_t n_tickets, uint2* reduced, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_aux, dim3(n_units), dim3(kMinmaxThreads), 0, stream, fields, units, tickets,
                       n_tickets);
    hipLaunchKernelGGL(k_batch_range, dim3(n_fields), dim3(64), 0, stream, fields, reduced);
}

void launch_batch_place(const PlaceField* fields, const uint2* units, uint32_t n_units, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_chunk_sums, dim3(n_units), dim3(256), 0, stream, fields, units);
    hipLaunchKernelGGL(k_batch_scatter, dim3(n_units * kChunkSplit), dim3(256), 0, stream, fields, units);
}

__global__ __launch_bounds__(256) void k_scatter_overflow(Staging stg, const Scalars* sc, const ResultDev* res,
                                                          const uint32_t* __restrict__ tile_off,
                                                          const uint32_t* __restrict__ block_info, Geom g,
                                                          uint32_t* __restrict__ out_idx,
                                                          int32_t* __restrict__ out_val) {
    const uint32_t ovf_n = min(sc->stage_count, stg.ovf_cap);
    if (blockIdx.x * blockDim.x >= ovf_n) return;
    if (load_status(&res->status) != ST_OK) return;
    const uint32_t n = (uint32_t)res->n_out;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ovf_n; i += gridDim.x * blockDim.x) {
        const uint4 e = stg.ovf[i];
        place_entry(e, tile_off[block_tile(e.z, g)], block_info, n, out_idx, out_val);
    }
}

void launch_chunked_place(const Staging& stg, const Scalars* sc, void* res, uint64_t out_cap,
                          const uint32_t* tile_count, uint32_t* tile_off, uint32_t* chunk_sum, uint32_t n_tiles,
                          const uint32_t* block_info, Geom g, uint32_t* out_idx, int32_t* out_val,
                          hipStream_t stream) {
    const uint32_t n_chunks = (n_tiles + kChunkTiles - 1) / kChunkTiles;
    hipLaunchKernelGGL(k_chunk_sums, dim3(n_chunks), dim3(256), 0, stream, tile_count, n_tiles, chunk_sum);
    hipLaunchKernelGGL(k_scatter_chunks, dim3(n_chunks * kChunkSplit), dim3(256), 0, stream, stg, (ResultDev*)res,
                       out_cap, tile_count, tile_off, (const uint32_t*)chunk_sum, n_tiles, n_chunks, block_info, g,
                       out_idx, out_val);
    if (stg.ovf_cap > 0 && !stg.dense)
        hipLaunchKernelGGL(k_scatter_overflow, dim3(1024), dim3(256), 0, stream, stg, sc, (const ResultDev*)res,
                           (const uint32_t*)tile_off, block_info, g, out_idx, out_val);
}

// ------------------------------------------------------------------ fused scan + scatter

// One kernel for fields of at most kPlaceTiles tiles. Workgroup w looks at
// the tiles t = w (mod grid) and its slice of the overflow list; if it has
// anything to place (and always for workgroup 0, which writes n_out and the
// capacity verdict) it computes the exclusive scan of all tile counts in LDS
// itself and places its share. With no outliers only workgroup 0 scans.
//
// The scan takes one round trip to L2: thread k loads the counts of tiles
// 4k .. 4k+3 of every 1024-tile pass as one uint4 (the count array is padded
// to 256 bytes, so reads up to the next multiple of 4 stay inside it; the
// entries past n_tiles are masked), all passes are scanned at once and one
// barrier publishes the per-wave sums.
__global__ __launch_bounds__(256) void k_place(Staging stg, const Scalars* sc, ResultDev* res, uint64_t out_cap,
                                               const uint32_t* __restrict__ tile_count, uint32_t n_tiles,
                                               const uint32_t* __restrict__ block_info, Geom g,
                                               uint32_t* __restrict__ out_idx, int32_t* __restrict__ out_val) {
    constexpr int kPasses = kPlaceTiles / 1024;
    __shared__ uint4 pre4[kPlaceTiles / 4];
    __shared__ uint32_t wsum[kPasses][4];
    const uint32_t* pre = reinterpret_cast<const uint32_t*>(pre4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t G = gridDim.x;
    const bool lead = blockIdx.x == 0;
    const uint32_t ovf_n = min(sc->stage_count, stg.ovf_cap);
    if (!lead) {
        bool mine = false;
        for (uint32_t t = blockIdx.x + (uint32_t)tid * G; t < n_tiles; t += 256u * G) mine = mine || tile_count[t] != 0;
        mine = __syncthreads_or(mine) || blockIdx.x * 256u < ovf_n;
        if (!mine) return;
    }
    const uint32_t n4 = (n_tiles + 3) / 4;
    const uint4* cnt4 = reinterpret_cast<const uint4*>(tile_count);
    uint4 v[kPasses];
#pragma unroll
    for (int j = 0; j < kPasses; ++j) v[j] = cnt4[min((uint32_t)tid + 256u * j, n4 - 1)];
    uint32_t s[kPasses], incl[kPasses];
#pragma unroll
    for (int j = 0; j < kPasses; ++j) {
        const uint32_t i = 4u * ((uint32_t)tid + 256u * j);
        if (i >= n_tiles) v[j].x = 0u;
        if (i + 1 >= n_tiles) v[j].y = 0u;
        if (i + 2 >= n_tiles) v[j].z = 0u;
        if (i + 3 >= n_tiles) v[j].w = 0u;
        s[j] = v[j].x + v[j].y + v[j].z + v[j].w;
        incl[j] = wave_scan_incl(s[j], lane);
        if (lane == 63) wsum[j][wave] = incl[j];
    }
    __syncthreads();
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < kPasses; ++j) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t ws = wsum[j][w];
            all += ws;
            before += w < wave ? ws : 0u;
        }
        const uint32_t run = carry + before + incl[j] - s[j];
        const uint32_t i4 = (uint32_t)tid + 256u * j;
        if (i4 < n4) {
            const uint32_t r1 = run + v[j].x, r2 = r1 + v[j].y;
            pre4[i4] = make_uint4(run, r1, r2, r2 + v[j].z);
        }
        carry += all;
    }
    const uint64_t total = carry;  // the outlier count is below the cell count, below 2^32
    if (lead && tid == 0 && load_status(&res->status) == ST_OK) {
        res->n_out = total;
        if (total > out_cap) store_status(&res->status, ST_ECAPACITY);
    }
    __syncthreads();
    if (total == 0 || total > out_cap || load_status(&res->status) != ST_OK) return;  // nothing, or incomplete
    const uint32_t n = (uint32_t)total;
    if (stg.dense) {
        for (uint32_t t = blockIdx.x + (uint32_t)wave * G; t < n_tiles; t += 4u * G) {
            const uint32_t c = tile_count[t];
            if (c) place_tile_dense(stg, g, t, pre[t], c, block_info, n, out_idx, out_val, lane);
        }
        return;
    }
    if (stg.spt) {
        for (uint32_t t = blockIdx.x + (uint32_t)wave * G; t < n_tiles; t += 4u * G) {
            const uint32_t c = min(tile_count[t], stg.spt);
            if (c == 0) continue;
            const uint4* reg = stg.region + (uint64_t)t * stg.spt;
            for (uint32_t i = (uint32_t)lane; i < c; i += 64) place_entry(reg[i], pre[t], block_info, n, out_idx, out_val);
        }
    }
    for (uint32_t i = blockIdx.x * 256u + tid; i < ovf_n; i += G * 256u) {
        const uint4 e = stg.ovf[i];
        place_entry(e, pre[block_tile(e.z, g)], block_info, n, out_idx, out_val);
    }
}

void launch_place(const Staging& stg, const Scalars* sc, void* res, uint64_t out_cap, const uint32_t* tile_count,
                  uint32_t n_tiles, const uint32_t* block_info, Geom g, uint32_t* out_idx, int32_t* out_val,
                  hipStream_t stream) {
    uint32_t blocks = (n_tiles + 3) / 4;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_place, dim3(blocks), dim3(256), 0, stream, stg, sc, (ResultDev*)res, out_cap,
                       tile_count, n_tiles, block_info, g, out_idx, out_val);
}

// ------------------------------------------------------------------ decompress

struct IndexGeom {
    Geom g;
    FastDiv dx, dy;  // by nx, by ny
    uint32_t lb;     // log2 B
};

// (block, local row-major position) of a cell as one 64-bit key: the list's
// order is the keys' order.
__device__ __forceinline__ uint64_t cell_key(const IndexGeom& ig, uint32_t idx) {
    const uint32_t rest = ig.dx.div(idx);
    const uint32_t x = idx - rest * ig.g.nx;
    const uint32_t z = ig.dy.div(rest);
    const uint32_t y = rest - z * ig.g.ny;
    const uint32_t bid = ((z >> ig.lb) * ig.g.nby + (y >> ig.lb)) * ig.g.nbx + (x >> ig.lb);
    const uint32_t m = (1u << ig.lb) - 1u;
    const uint32_t local = (((z & m) << ig.lb | (y & m)) << ig.lb) | (x & m);
    return ((uint64_t)bid << 32) | local;
}

// First position in [lo, hi) of the outlier list whose block is >= b (hi if
// none); an index outside the field counts as past every block.
__device__ __forceinline__ uint32_t first_at_or_after(const uint32_t* __restrict__ out_idx, uint32_t lo, uint32_t hi,
                                                      uint32_t b, const IndexGeom& ig) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        const uint32_t idx = out_idx[mid];
        const uint32_t bb = idx < ig.g.N ? (uint32_t)(cell_key(ig, idx) >> 32) : 0xffffffffu;
        if (bb < b) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr uint32_t kIndexGrid = 4096;  // workgroups at most; both loops stride over the grid
constexpr int kIndexUnroll = 4;        // list entries per lane per step (loads in flight together)

// block_start[b] = first outlier of block b or later (b = 0..n_blocks);
// outliers must be in strictly increasing (block, local row-major) order,
// else the call's status becomes DQ_ECORRUPT.
__global__ __launch_bounds__(256) void k_index(const uint32_t* __restrict__ out_idx, uint32_t n_out,
                                               IndexGeom ig, uint32_t* __restrict__ block_start,
                                               unsigned long long* res_word, uint32_t tag,
                                               const ResultView* src, uint32_t cap) {
    const int lane = threadIdx.x & 63;
    const uint64_t N = ig.g.N;
    if (src) {  // the count of the compress call that wrote the list (at most its capacity)
        const unsigned long long n = src->n_out;
        n_out = (uint32_t)(n < cap ? n : cap);
    }
    // order check: each wave takes kIndexUnroll x 64 consecutive entries per
    // step; an entry's predecessor key comes from the lane below, lane 0 of a
    // piece takes lane 63 of the piece before, the wave's first entry loads
    // its predecessor. A key of ~0 marks an index outside the field.
    constexpr uint64_t kBad = ~0ull;
    const uint32_t wave_step = kIndexUnroll * 64u;
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    bool bad = false;
    for (uint64_t base = (uint64_t)wave_id * wave_step; base < n_out; base += (uint64_t)n_waves * wave_step) {
        uint32_t idx[kIndexUnroll];
#pragma unroll
        for (int u = 0; u < kIndexUnroll; ++u) {
            const uint64_t i = base + (uint64_t)u * 64u + (uint64_t)lane;
            idx[u] = i < n_out ? out_idx[i] : 0u;
        }
        uint32_t before = 0;
        if (lane == 0 && base > 0) before = out_idx[base - 1];
        uint64_t carry = (base > 0 && before < N) ? cell_key(ig, before) : kBad;
#pragma unroll
        for (int u = 0; u < kIndexUnroll; ++u) {
            const uint64_t i = base + (uint64_t)u * 64u + (uint64_t)lane;
            const bool in = i < n_out;
            const uint64_t key = (in && idx[u] < N) ? cell_key(ig, idx[u]) : kBad;
            const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
            uint64_t prev = ((uint64_t)(uint32_t)__shfl_up((int)hi, 1) << 32) | (uint32_t)__shfl_up((int)lo, 1);
            if (lane == 0) prev = carry;
            if (in) bad |= key == kBad || (i > 0 && !(prev < key));
            carry = ((uint64_t)readlane(hi, 63) << 32) | readlane(lo, 63);
        }
    }
    if (bad) status_corrupt_tagged(res_word, tag);
    // block_start of 256 blocks per workgroup step: two searches over the
    // list bound the range in which all of them lie, then every thread
    // searches that (short, cache-resident) range
    __shared__ uint32_t range[2];
    const uint32_t nb1 = ig.g.nblocks + 1;
    uint32_t from = 0;
    for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < nb1; b0 += gridDim.x * blockDim.x) {  // uniform in the workgroup
        if (threadIdx.x < 2) {
            const uint32_t target = threadIdx.x == 0 ? b0 : min(b0 + blockDim.x, nb1);
            range[threadIdx.x] = first_at_or_after(out_idx, from, n_out, target, ig);
        }
        __syncthreads();
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t r0 = range[0], r1 = range[1];
        if (b < nb1) block_start[b] = first_at_or_after(out_idx, r0, r1, b, ig);
        from = r1;  // later steps look at later blocks
        __syncthreads();
    }
}

void launch_index(const uint32_t* out_idx, uint32_t n_out, Geom g, int block_log2, int dim,
                  uint32_t* block_start, void* res, uint32_t tag, hipStream_t stream, const void* src,
                  uint32_t cap) {
    (void)dim;
    IndexGeom ig{g, make_fastdiv(g.nx), make_fastdiv(g.ny), (uint32_t)block_log2};
    const uint64_t cnt = src ? (uint64_t)cap : (uint64_t)n_out;  // with src: the largest possible count
    const uint64_t list_groups = (cnt + 4u * kIndexUnroll * 64u - 1) / (4u * kIndexUnroll * 64u);
    const uint64_t block_groups = ((uint64_t)g.nblocks + 1 + 255) / 256;
    uint64_t blocks = list_groups > block_groups ? list_groups : block_groups;
    if (blocks > kIndexGrid) blocks = kIndexGrid;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_index, dim3((uint32_t)blocks), dim3(256), 0, stream, out_idx, n_out, ig, block_start,
                       reinterpret_cast<unsigned long long*>(res), tag, (const ResultView*)src, cap);
}

// Clears a result's status word (tag 0 is never a call's tag), so that a
// decompress enqueued again with the same tag (a replayed graph) starts clean.
__global__ void k_result_reset(unsigned long long* w) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *w = 0ull;
}

void launch_result_reset(void* res, hipStream_t stream) {
    hipLaunchKernelGGL(k_result_reset, dim3(1), dim3(64), 0, stream, reinterpret_cast<unsigned long long*>(res));
}

}  // namespace dq
