// dq_device.hpp - shared device helpers of libdq (gfx950, wave64).
//
// Tiling. The field is cut into cubic blocks of edge B (Section III-A: SZ
// compresses fixed-size blocks independently). A wave owns a "tile": a run of
// consecutive blocks along x inside one block row (fixed block indices along
// y and z), so a tile covers a contiguous range of block ids. Lanes span x:
// lane l holds V consecutive x cells, the wave covers CX = 64*V cells of one
// grid row per step, and a block row segment is GPB = B/V lanes wide. The
// wave walks the block's rows (y, then z) in local row-major order, carrying
// the previous row (and, in 3-D, the previous plane) in registers, so every
// grid row is read once with fully coalesced 4V-byte loads and the codes are
// written with 2V-byte stores. When B > CX (1-D only) a block spans several
// steps and the x neighbour of lane 0 is carried across steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dq {

constexpr int kWaves = 4;                 // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kStageCap = 256;            // LDS outlier staging entries per wave
constexpr uint32_t kOriginFlag = 0x80000000u;
constexpr int kTileTarget = 1024;         // minimum cells per tile (1-D, 2-D)

// The dispatcher hands the workgroups of a launch to the 8 XCDs in turn
// (workgroup i to XCD i mod 8), and every XCD has an L2 of its own. Tile
// kernels renumber their workgroups so that each XCD receives one contiguous
// range of tiles: neighbouring tiles of a row, which share cache lines
// whenever a row is not a whole number of 128-byte lines, are then read and
// written through one L2 instead of two (a bijection of [0, n)).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n) {
    const uint32_t x = b % kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

constexpr int ST_OK = 0, ST_EINVAL = -1, ST_ERANGE = -2, ST_ECAPACITY = -3, ST_ECORRUPT = -6;
constexpr int PAD_ZERO = 0, PAD_BLOCK = 1, PAD_EDGE = 2, PAD_GLOBAL = 3;
constexpr int PAD_BLOCK_MIN = 4, PAD_BLOCK_MAX = 5, PAD_GLOBAL_MIN = 6, PAD_GLOBAL_MAX = 7;
constexpr int PAD_GIVEN = 8;  // per-block values supplied by the caller (read by encode)
// one stored value per block / per field
__host__ __device__ constexpr bool pad_per_block(int m) {
    return m == PAD_BLOCK || m == PAD_BLOCK_MIN || m == PAD_BLOCK_MAX || m == PAD_GIVEN;
}
__host__ __device__ constexpr bool pad_global(int m) {
    return m == PAD_GLOBAL || m == PAD_GLOBAL_MIN || m == PAD_GLOBAL_MAX;
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Batches of rows kept in flight ahead of the one being computed (interior
// tiles; see k_encode / k_decode) and the most grid rows of a block row that
// are unrolled into straight-line code.
#ifndef DQ_PIPE_DEPTH
#define DQ_PIPE_DEPTH 3
#endif
constexpr int kPipeDepth = DQ_PIPE_DEPTH;
constexpr int kMaxUnrollRows = 64;

template <int I>
struct Idx {
    static constexpr int value = I;
};

// f(Idx<I>{}) for I = FIRST .. LAST-1, expanded at compile time
template <int FIRST, int LAST, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (FIRST < LAST) {
        f(Idx<FIRST>{});
        static_for<FIRST + 1, LAST>(f);
    }
}

template <int DIM, int B, int V>
struct Cfg {
    static constexpr int CX = 64 * V;                       // cells per wave step
    static constexpr bool WIDE = B > CX;                    // block spans steps (1-D)
    static constexpr int GPB = WIDE ? 64 : B / V;           // lanes per block row
    static constexpr int BPC = WIDE ? 1 : CX / B;           // blocks per step
    static constexpr int NCH = WIDE ? B / CX : 1;           // steps per block row
    static constexpr int BY = DIM >= 2 ? B : 1;
    static constexpr int BZ = DIM == 3 ? B : 1;
    static constexpr int XCH = WIDE ? 1 : cmax(1, kTileTarget / (CX * BY * BZ));
    static constexpr int BPT = WIDE ? cmax(1, kTileTarget / B) : XCH * BPC;  // blocks per tile
    // rows whose loads are issued together before any is used (a batch): in
    // 3-D a whole block plane or half of it (at most 32 registers of cells
    // per lane), up to 8 rows in 2-D, up to 8 wave steps in 1-D
    static constexpr int NBR = WIDE ? cmin(NCH, 8)
                                    : (DIM == 3 ? cmin(BY, 32 / V) : (DIM == 2 ? cmin(BY, 8) : cmin(XCH, 8)));
    static_assert(DIM != 3 || BY == NBR || BY == 2 * NBR, "3-D batches cover a plane or half of it");
    // batches per block row of a complete block (2-D / 3-D)
    static constexpr int NBT = DIM == 3 ? BZ * (BY / NBR) : (DIM == 2 ? BY / NBR : 1);
    static_assert(V == 1 || V == 2 || V == 4, "V");
    static_assert(V <= B, "V <= B");
    static_assert(!WIDE || DIM == 1, "only 1-D blocks may be wider than a wave step");
    static_assert(DIM < 3 || B * V <= 64, "3-D plane carry must fit in registers");
};

// Field geometry (x fastest). Unused axes have extent 1 and one block.
struct Geom {
    uint32_t nx, ny, nz;
    uint32_t nbx, nby, nbz;
    uint32_t ntx;      // tiles per block row
    uint32_t bpt;      // blocks per tile along x
    uint32_t n_tiles;
    uint32_t nblocks;
    uint64_t N;
};

// Device scalars of one compress call (at the start of the workspace).
struct Scalars {
    double eb;             // absolute error bound
    double twoeb;          // 2 eb
    double r;              // fp64 reciprocal of 2 eb (first estimate only)
    unsigned long long sumq;   // int64 sum of q, two's complement (GLOBAL pad)
    unsigned int stage_count;  // entries appended to the overflow staging list
    int gpad;                  // global pad value
};

// The error bound of a compress call as the kernels receive it: either the
// absolute bound itself, or the relative factor and the per-workgroup
// partials of the value-range pass (min key, max key; a max key of all ones
// marks a non-finite input, since no finite or infinite value maps to it),
// which each wave of the consuming kernel reduces itself.
struct BoundArgs {
    const uint2* parts;  // always a valid, 16-byte aligned address of kBoundParts entries
    int nparts;          // value-range partials (0: no value-range pass)
    double v;            // absolute bound, or the relative factor
    int rel;             // 1: eb = v * (max - min) over the partials
};

// Staging of the outliers found by the encode pass, in the compress
// workspace: every tile owns a region of spt slots (written without atomics);
// what does not fit goes to an overflow list, appended with one atomic per
// flush. Entries are (C-order index, delta, block id, rank among the block's
// non-origin outliers | kOriginFlag for the origin) and say where they go,
// so the order inside the staging area does not matter.
struct Staging {
    uint4* region;     // n_tiles * spt entries
    uint32_t spt;      // slots per tile (may be 0)
    uint4* ovf;        // overflow list
    uint32_t ovf_cap;
    // dense: a tile's region holds a slot for every cell (2 spt >= cells per
    // tile): its region is an array of uint2 (index, residual) where block j
    // of the tile owns slots j * bcells .. (j + 1) * bcells - 1, its origin
    // at the first, the non-origin outlier of rank r at 1 + r; the encode
    // writes every outlier there directly (no LDS staging, no overflow)
    uint32_t dense;
    uint32_t bcells;   // cells per block (B^d)
};

struct EncArgs {
    BoundArgs bound;
    double* eb_out;        // dq_result.eb_abs (written for a relative bound)
    const float* x;
    uint16_t* codes;
    int32_t* pads;
    uint32_t* block_info;  // per block: outliers of earlier blocks in the tile | origin flag
    uint32_t* tile_count;  // per tile: outliers in the tile
    Staging stg;
    Scalars* sc;
    int32_t* status;       // dq_result.status
    Geom g;
    int32_t R;
    int32_t pad_mode;
};

// Status of a decompress call, initialised by the decode kernel itself: the
// first 8 bytes of dq_result (status, reserved) form one word whose upper
// half carries the call's tag. Tile 0 sets (tag, OK) unless the word already
// holds this call's tag; a corruption report sets (tag, ECORRUPT)
// unconditionally. Either order leaves ECORRUPT if any report was made.
__device__ __forceinline__ void status_init_tagged(unsigned long long* w, uint32_t tag) {
    unsigned long long old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long ok = ((unsigned long long)tag << 32) | (uint32_t)ST_OK;
    while ((uint32_t)(old >> 32) != tag) {
        if (__hip_atomic_compare_exchange_strong(w, &old, ok, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            break;
    }
}

__device__ __forceinline__ void status_corrupt_tagged(unsigned long long* w, uint32_t tag) {
    (void)__hip_atomic_exchange(w, ((unsigned long long)tag << 32) | (uint32_t)ST_ECORRUPT, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}

// Read-only view of a dq_result written by an earlier compress call.
struct ResultView {
    int32_t status;
    uint32_t reserved;
    unsigned long long n_out;
    double eb_abs;
};

__device__ __forceinline__ void status_set_tagged(unsigned long long* w, uint32_t tag, int st) {
    (void)__hip_atomic_exchange(w, ((unsigned long long)tag << 32) | (uint32_t)st, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}

struct DecArgs {
    const ResultView* src;         // non-null: n_out / eb_abs come from this compress result
    uint32_t cap;                  // with src: the out_cap of that compress call
    unsigned long long* res_word;  // dq_result status + reserved (tagged, see above)
    unsigned long long* n_out_out; // dq_result.n_out
    double* eb_out;                // dq_result.eb_abs
    double eb_abs;
    uint32_t tag;
    const uint16_t* codes;
    const uint32_t* out_idx;
    const int32_t* out_val;
    const int32_t* pads;
    const uint32_t* block_start;  // n_blocks + 1 entries (unused when n_out == 0), or NULL:
    // then the runs come from the compress call's tile offsets (tile_off),
    // tile counts and in-tile block prefixes (block_info) - decoding in the
    // same batch as the compress, with the compress call's tiling
    const uint32_t* tile_off;
    const uint32_t* tile_count;
    const uint32_t* block_info;
    float* x_hat;
    Geom g;
    double twoeb;
    uint32_t n_out;
    int32_t R;
    int32_t pad_mode;
};

// First and one-past-last outlier of block blk.
__device__ __forceinline__ void block_run(const DecArgs& a, uint32_t blk, uint32_t& os, uint32_t& oe) {
    if (a.block_start) {
        os = a.block_start[blk];
        oe = a.block_start[blk + 1];
        return;
    }
    const uint32_t bx = blk % a.g.nbx, row = blk / a.g.nbx;
    const uint32_t t = row * a.g.ntx + bx / a.g.bpt;
    const uint32_t base = a.tile_off[t];
    os = base + (a.block_info[blk] & ~kOriginFlag);
    const bool last = (bx + 1) % a.g.bpt == 0 || bx + 1 == a.g.nbx;
    oe = base + (last ? a.tile_count[t] : (a.block_info[blk + 1] & ~kOriginFlag));
}

// Work queue of a persistent batch kernel: units of consecutive tiles of one
// field, taken in ticket order; the arguments of every field of the batch.
struct BatchQueue {
    const EncArgs* enc;
    const DecArgs* dec;
    const uint4* units;  // (field, first tile, tiles, 0)
    uint32_t n_units;
    unsigned int* ticket;
};

// ------------------------------------------------------------------ lanes

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of m in lanes below this lane
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }

// value of lane-1 (lane 0 receives 0): DPP wave_shr:1. The empty asm keeps
// the shifted value in a register of its own: folded into a subtraction
// `x - shifted`, this compiler emits v_subrev_u32_dpp, which on gfx950
// returned shifted - x (checked on the device; v_sub/v_add with DPP and a
// DPP move were correct).
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v) {
    uint32_t s = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);
    __asm__("" : "+v"(s));
    return s;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// A DPP move inside rows of 16 lanes (every source lane exists), kept in a
// register of its own like wave_shr1.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_row(uint32_t v) {
    uint32_t s = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
    __asm__("" : "+v"(s));
    return s;
}

// Minimum / maximum over the whole wave (all lanes active), returned as a
// scalar: quad swaps, then the half-row and row mirrors leave every row of 16
// lanes holding its extreme; the four rows' values are read with readlane.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, dpp_row<0xB1>(v));   // quad_perm [1, 0, 3, 2]
    v = min(v, dpp_row<0x4E>(v));   // quad_perm [2, 3, 0, 1]
    v = min(v, dpp_row<0x141>(v));  // row_half_mirror
    v = min(v, dpp_row<0x140>(v));  // row_mirror
    return min(min(readlane(v, 0), readlane(v, 16)), min(readlane(v, 32), readlane(v, 48)));
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_row<0xB1>(v));
    v = max(v, dpp_row<0x4E>(v));
    v = max(v, dpp_row<0x141>(v));
    v = max(v, dpp_row<0x140>(v));
    return max(max(readlane(v, 0), readlane(v, 16)), max(readlane(v, 32), readlane(v, 48)));
}

// a value every lane holds identically, kept in a scalar register
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ double uniform(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = uniform((uint32_t)u), hi = uniform((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}

// Inclusive prefix sum of v over aligned segments of G lanes (G power of 2).
template <int G>
__device__ __forceinline__ uint32_t seg_scan_incl(uint32_t v, int lane) {
    if constexpr (G >= 2) {
        uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
        v += ((lane & (G - 1)) >= 1) ? t : 0u;
    }
    if constexpr (G >= 4) {
        uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
        v += ((lane & (G - 1)) >= 2) ? t : 0u;
    }
    if constexpr (G >= 8) {
        uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
        v += ((lane & (G - 1)) >= 4) ? t : 0u;
    }
    if constexpr (G >= 16) {
        uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
        v += ((lane & 15) >= 8) ? t : 0u;
    }
    if constexpr (G >= 32) {
        // lane 15 of rows 0 and 2 -> rows 1 and 3
        uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
        v += t;
    }
    if constexpr (G >= 64) {
        // lane 31 -> rows 2 and 3
        uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
        v += t;
    }
    return v;
}

// Minimum / maximum over aligned groups of G lanes.
template <int G>
__device__ __forceinline__ int32_t group_min32(int32_t v) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) v = min(v, __shfl_xor(v, off));
    return v;
}
template <int G>
__device__ __forceinline__ int32_t group_max32(int32_t v) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// Sum over aligned groups of G lanes (every lane of a group gets the sum).
template <int G>
__device__ __forceinline__ long long group_sum64(long long v) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

// Inclusive prefix sum over the whole wave (rare paths only).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// ------------------------------------------------------------------ arithmetic

// Nearest integer to S / n (n > 0), exact halves toward +infinity.
__device__ __forceinline__ int32_t round_mean(long long S, long long n) {
    long long q = S / n;
    long long rm = S - q * n;
    if (rm < 0) {
        q -= 1;
        rm += n;
    }
    return (int32_t)(q + ((2 * rm >= n) ? 1 : 0));
}

// Effective padding of a block: sum over non-empty axis sets S of
// (-1)^(|S|+1) * halo(S). Constant halos give the pad itself; EDGE halos use
// the per-axis values e[a] and rounded means for cells in front along
// several axes.
template <int DIM>
__device__ __forceinline__ uint32_t edge_effective(const int32_t* e) {
    if constexpr (DIM == 1) {
        return (uint32_t)e[0];
    } else if constexpr (DIM == 2) {
        long long s = (long long)e[0] + e[1];
        return (uint32_t)(s - round_mean(s, 2));
    } else {
        long long s01 = (long long)e[0] + e[1], s02 = (long long)e[0] + e[2], s12 = (long long)e[1] + e[2];
        long long s = s01 + e[2];
        long long v = s - round_mean(s01, 2) - round_mean(s02, 2) - round_mean(s12, 2) + round_mean(s, 3);
        return (uint32_t)v;
    }
}

// Pre-quantisation (Section III-A): q = nearest integer to x / (2 eb), exact
// halves to even. Fast path: k = rint(x * r) with r = fl(1 / (2 eb)); k is
// exact unless x*r lies within 2^-16 of a half-integer (its error is below
// 2^-18 while |x*r| < 2^32). Near halves the exact residual e = x - 2 eb k is
// obtained with one fma (its comparison with +-eb is exact) and k is moved by
// one if needed. The caller runs the slow path for the whole wave when any
// lane needs it.
constexpr double kNearHalf = 0.5 - 1.52587890625e-05;  // 0.5 - 2^-16
constexpr double kQMax = 2147483647.0;
constexpr double kRoundShift = 6755399441055744.0;  // 1.5 * 2^52

__device__ __forceinline__ double exact_round(float x, double k, double twoeb, double eb) {
    const double e = __builtin_fma(-twoeb, k, (double)x);
    if (e > eb) return k + 1.0;
    if (e < -eb) return k - 1.0;
    if (e == eb || e == -eb) {
        const double h = k * 0.5;
        if (h != __builtin_rint(h)) return e > 0.0 ? k + 1.0 : k - 1.0;  // odd: go to the even side
    }
    return k;
}

// `bad` accumulates (wave-wide) lanes whose q is out of range or x is not
// finite. The fast path needs |x*r| <= 2^31 - 1.5 (then |q| <= 2^31 - 1
// for sure) and x*r away from a half; every other lane - near a half, near or
// past the range limit, non-finite - sends the wave through the exact path.
constexpr double kFastMax = 2147483646.5;

template <int V>
__device__ __forceinline__ void prequant(const float (&x)[V], double r, double twoeb, double eb,
                                         uint32_t (&q)[V], uint64_t& bad) {
    double k[V];
    bool slow = false;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const double v = (double)x[j] * r;
        k[j] = __builtin_rint(v);
        // false for NaN, so a non-finite x also takes the exact path
        const bool fast = __builtin_fabs(v - k[j]) <= kNearHalf && __builtin_fabs(v) <= kFastMax;
        slow = slow || !fast;
    }
    if (__builtin_expect(ballot(slow) != 0, 0)) {
        bool out = false;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            k[j] = exact_round(x[j], k[j], twoeb, eb);
            out = out || !(__builtin_fabs(k[j]) <= kQMax);  // NaN and +-inf fail too
            k[j] = __builtin_fabs(k[j]) <= kQMax ? k[j] : 0.0;
        }
        bad |= ballot(out);
    }
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = (uint32_t)(int32_t)k[j];
}

// ------------------------------------------------------------------ error bound

// order-preserving map of a finite float to uint32, and back
__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float funkey(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

struct Bound {
    double eb, twoeb, r;
    float mn, mx;  // value range of the field (with the value-range pass)
    int status;    // ST_OK, ST_ERANGE (non-finite input), ST_EINVAL (zero value range)
};

// At most kBoundParts value-range partials (the value-range pass launches at
// most that many workgroups), read by a wave as 16-byte pairs, kBoundLoads
// per lane.
constexpr int kBoundParts = 256;
constexpr int kBoundLoads = kBoundParts / 128;

// Issue the loads of the partials (every lane loads, from the valid address
// even for an absolute bound, so no path skips them; entries past nparts are
// ignored); bound_finish waits.
__device__ __forceinline__ void bound_fetch(const BoundArgs& b, uint4 (&pp)[kBoundLoads], int lane) {
    const uint4* p2 = reinterpret_cast<const uint4*>(b.parts);
    if (b.nparts > 2) {
#pragma unroll
        for (int k = 0; k < kBoundLoads; ++k) pp[k] = p2[lane + 64 * k];
    } else {  // one pair (a batch's pre-reduced value range): one 16-byte load
        pp[0] = p2[0];
#pragma unroll
        for (int k = 1; k < kBoundLoads; ++k) pp[k] = make_uint4(0u, 0u, 0u, 0u);
    }
}

// The absolute bound, resolved for a relative one (Section II-B, value-range
// relative bound): eb = rel * (max - min) over the finite inputs. Wave-wide
// (no barrier); every lane gets the same result.
__device__ __forceinline__ Bound bound_finish(const BoundArgs& b, const uint4 (&pp)[kBoundLoads], int lane) {
    Bound o;
    o.status = ST_OK;
    o.mn = o.mx = 0.0f;
    o.eb = b.v;
    if (b.nparts != 0) {
        uint32_t kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
        for (int k = 0; k < kBoundLoads; ++k) {
            const int i = 2 * (lane + 64 * k);  // partials i (x, y) and i + 1 (z, w)
            kmin = i < b.nparts ? min(kmin, pp[k].x) : kmin;
            kmax = i < b.nparts ? max(kmax, pp[k].y) : kmax;
            kmin = i + 1 < b.nparts ? min(kmin, pp[k].z) : kmin;
            kmax = i + 1 < b.nparts ? max(kmax, pp[k].w) : kmax;
        }
        kmin = wave_min_u32(kmin);
        kmax = wave_max_u32(kmax);
        const bool nf = kmax == 0xffffffffu;
        o.mn = __uint_as_float(uniform(__float_as_uint(funkey(kmin))));
        o.mx = __uint_as_float(uniform(__float_as_uint(funkey(kmax))));
        if (b.rel) o.eb = b.v * ((double)o.mx - (double)o.mn);
        if (nf) {
            o.status = ST_ERANGE;
        } else if (b.rel &&
                   (!(o.eb > 0.0) || !__builtin_isfinite(o.eb) || !__builtin_isfinite(1.0 / (2.0 * o.eb)))) {
            o.status = ST_EINVAL;
        }
    }
    if (o.status != ST_OK && b.rel) o.eb = 0.0;
    o.eb = uniform(o.eb);  // wave-uniform: keep the bound in scalar registers
    o.status = (int)uniform((uint32_t)o.status);
    o.twoeb = 2.0 * o.eb;
    o.r = o.status == ST_OK ? 1.0 / (2.0 * o.eb) : 0.0;
    o.r = uniform(o.r);
    return o;
}

// ------------------------------------------------------------------ vector memory

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int V>
__device__ __forceinline__ void load_f(const float* p, float (&v)[V]) {
    if constexpr (V == 1) {
        v[0] = __builtin_nontemporal_load(p);
    } else if constexpr (V == 2) {
        f32x2 t = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p));
        v[0] = t.x; v[1] = t.y;
    } else {
        f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
}

template <int V>
__device__ __forceinline__ void store_f(float* p, const float (&v)[V]) {
    if constexpr (V == 1) {
        __builtin_nontemporal_store(v[0], p);
    } else if constexpr (V == 2) {
        f32x2 t = {v[0], v[1]};
        __builtin_nontemporal_store(t, reinterpret_cast<f32x2*>(p));
    } else {
        f32x4 t = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(t, reinterpret_cast<f32x4*>(p));
    }
}

// Codes are stored with the default (write-back) cache policy, and loaded
// with it wherever a row of codes may not start on a 128-byte line. Such a
// row shares its first and last lines with the neighbouring tiles' rows:
// write-through stores sent each part of a shared line to memory on its own
// (a partial-line write), and nontemporal loads did not keep the line in the
// L2 for the neighbour, so it was fetched twice (on rows of 450 or 480 cells
// the decode took 45-65 % longer, the encode up to 25 %). Fields whose rows
// all start on lines are decoded with nontemporal loads, which leave the L2
// and the Infinity Cache to the data that is read again.
// V uint16 codes, packed in 16-bit halves of 32-bit words
template <int V>
__device__ __forceinline__ void store_codes(uint16_t* p, const uint32_t (&c)[V]) {
    if constexpr (V == 1) {
        *p = (uint16_t)c[0];
    } else if constexpr (V == 2) {
        *reinterpret_cast<uint32_t*>(p) = c[0] | (c[1] << 16);
    } else {
        const uint64_t w = (uint64_t)(c[0] | (c[1] << 16)) | ((uint64_t)(c[2] | (c[3] << 16)) << 32);
        *reinterpret_cast<uint64_t*>(p) = w;
    }
}

// NT: nontemporal loads (see the note on codes above for when they are not)
template <int V, bool NT = false>
__device__ __forceinline__ void load_codes(const uint16_t* p, uint32_t (&c)[V]) {
    if constexpr (V == 1) {
        if constexpr (NT) c[0] = __builtin_nontemporal_load(p);
        else c[0] = *p;
    } else if constexpr (V == 2) {
        uint32_t w;
        if constexpr (NT) w = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
        else w = *reinterpret_cast<const uint32_t*>(p);
        c[0] = w & 0xffffu; c[1] = w >> 16;
    } else {
        u32x2 w;
        if constexpr (NT) w = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
        else w = *reinterpret_cast<const u32x2*>(p);
        c[0] = w.x & 0xffffu; c[1] = w.x >> 16; c[2] = w.y & 0xffffu; c[3] = w.y >> 16;
    }
}

// ------------------------------------------------------------------ buffer addressing
//
// Interior tiles address their rows through one buffer resource per tile
// (base = the tile's first cell): the row offset is a scalar (soffset) and
// the lane offset one vector register shared by every row, instead of one
// 64-bit address per row. Raw buffer, 32-bit data format, no bounds beyond
// 2^31 - 1 bytes (the interior path requires the tile to span less).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcFlags = 0x00020000;
constexpr int kPolNT = 2;   // nontemporal
constexpr int kPolDefault = 0;  // codes (see store_codes)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A lane offset past the resource's range (2^31 - 1 bytes): a raw buffer
// access there is dropped by the hardware (a store writes nothing). Tiles
// that reach past the field's end store through it for their lanes and rows
// outside the field, so their stores stay unconditional like an interior
// tile's. The scalar row offset added to it stays below 2^31 - 1 wherever
// it is used (the pipelined path's tile-span bound), so the sum cannot wrap
// back into range.
constexpr uint32_t kOutOfRange = 0x80000000u;

__device__ __forceinline__ Rsrc make_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, kRsrcFlags);
}

template <int V>
__device__ __forceinline__ void load_f_buf(Rsrc rs, uint32_t voff, uint32_t soff, float (&v)[V]) {
    if constexpr (V == 1) {
        v[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, kPolNT));
    } else if constexpr (V == 2) {
        // reinterpret the whole vector as floats: splitting it into integer
        // lanes first made this compiler keep only the first dword of the load
        const f32x2 t = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, kPolNT));
        v[0] = t.x;
        v[1] = t.y;
    } else {
        const f32x4 t = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, kPolNT));
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
}

template <int V, int POL = kPolNT>
__device__ __forceinline__ void store_f_buf(Rsrc rs, uint32_t voff, uint32_t soff, const float (&v)[V]) {
    if constexpr (V == 1) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v[0]), rs, (int)voff, (int)soff, POL);
    } else if constexpr (V == 2) {
        const u32x2 t = {__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1])};
        __builtin_amdgcn_raw_buffer_store_b64(t, rs, (int)voff, (int)soff, POL);
    } else {
        const u32x4 t = {__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1]),
                         __builtin_bit_cast(uint32_t, v[2]), __builtin_bit_cast(uint32_t, v[3])};
        __builtin_amdgcn_raw_buffer_store_b128(t, rs, (int)voff, (int)soff, POL);
    }
}

// A lane of a decoded row segment whose 128-byte line the neighbouring
// segment also writes (the next tile, or the next row): the segment starts or
// ends inside that line. lo / hi: low 32 bits of the byte addresses of the
// segment's first byte and of its end.
__device__ __forceinline__ bool shares_line(uint32_t addr, uint32_t lo, uint32_t hi) {
    const uint32_t l = addr & ~127u;
    return (int32_t)(l - lo) < 0 || (int32_t)(hi - (l + 128u)) < 0;
}

template <int V>
__device__ __forceinline__ void store_codes_buf(Rsrc rs, uint32_t voff, uint32_t soff, const uint32_t (&c)[V]) {
    if constexpr (V == 1) {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)c[0], rs, (int)voff, (int)soff, kPolDefault);
    } else if constexpr (V == 2) {
        __builtin_amdgcn_raw_buffer_store_b32(c[0] | (c[1] << 16), rs, (int)voff, (int)soff, kPolDefault);
    } else {
        const u32x2 w = {c[0] | (c[1] << 16), c[2] | (c[3] << 16)};
        __builtin_amdgcn_raw_buffer_store_b64(w, rs, (int)voff, (int)soff, kPolDefault);
    }
}

template <int V, bool NT = false>
__device__ __forceinline__ void load_codes_buf(Rsrc rs, uint32_t voff, uint32_t soff, uint32_t (&c)[V]) {
    if constexpr (V == 1) {
        c[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)voff, (int)soff, NT ? kPolNT : kPolDefault);
    } else if constexpr (V == 2) {
        const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, NT ? kPolNT : kPolDefault);
        c[0] = w & 0xffffu;
        c[1] = w >> 16;
    } else {
        const u32x2 w = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, NT ? kPolNT : kPolDefault));
        c[0] = w.x & 0xffffu;
        c[1] = w.x >> 16;
        c[2] = w.y & 0xffffu;
        c[3] = w.y >> 16;
    }
}

// Move a wave's n LDS-staged outliers of tile t out of LDS: into the
// tile's region while it has room (placed = slots already used), the rest to
// the overflow list. Entries beyond the overflow capacity are dropped; that
// only happens when the outliers exceed the caller's capacity (ECAPACITY).
__device__ __forceinline__ void flush_stage(const uint4* sbuf, uint32_t n, const Staging& stg, uint32_t t,
                                            uint32_t& placed, unsigned int* counter, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t k = min(n, stg.spt - placed);
    uint4* reg = stg.region + (uint64_t)t * stg.spt + placed;
    for (uint32_t i = (uint32_t)lane; i < k; i += 64) reg[i] = sbuf[i];
    placed += k;
    const uint32_t rest = n - k;
    if (rest) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(counter, rest);
        base = readlane(base, 0);
        for (uint32_t i = (uint32_t)lane; i < rest; i += 64) {
            if ((uint64_t)base + i < stg.ovf_cap) stg.ovf[base + i] = sbuf[k + i];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Final position of a staged outlier of tile t whose tile offset in the
// list is off: the outliers of earlier blocks of the tile, then the block's
// origin (if it is an outlier) and the other outliers in local row-major
// order. Positions at or past n are not written.
__device__ __forceinline__ void place_entry(const uint4 e, uint32_t off, const uint32_t* block_info, uint32_t n,
                                            uint32_t* out_idx, int32_t* out_val) {
    const uint32_t info = block_info[e.z];
    uint32_t pos = off + (info & ~kOriginFlag);
    if (!(e.w & kOriginFlag)) pos += (info >> 31) + e.w;
    if (pos < n) {
        out_idx[pos] = e.x;
        out_val[pos] = (int32_t)e.y;
    }
}

__device__ __forceinline__ uint32_t block_tile(uint32_t b, const Geom& g) {
    const uint32_t bx = b % g.nbx;
    const uint32_t rest = b / g.nbx;
    const uint32_t by = rest % g.nby;
    const uint32_t bz = rest / g.nby;
    return (bz * g.nby + by) * g.ntx + bx / g.bpt;
}

}  // namespace dq
