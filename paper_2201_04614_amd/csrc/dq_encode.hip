// dq_encode.hip - fused dual-quantisation encode kernel (gfx950).
//
// One pass over x per tile (see dq_device.hpp for the tiling). Rows are
// handled in batches whose loads are all in flight before the first use, the
// next batch loading while the current one is computed:
//   q = round(x / 2eb)                                                (Section III-A)
//   -> zero-padded Lorenzo difference along x (DPP wave_shr:1), then y and z
//      against the previous row / plane kept in registers
//   -> code = delta + R or 0                                          (Section III-A)
//   -> uint16 stores; outliers found with ballots, ranked inside their block
//      and staged in LDS, flushed to a global staging list
//   -> at the end of each block: padding statistics (Section IV), the origin
//      residual q_o - P_eff (the only residual that depends on the padding,
//      because a face-constant halo cancels in every other Lorenzo
//      difference), per-block outlier bookkeeping.
// Inside a batch every phase is branch-free across rows; the two rare paths
// (exact rounding near halves, outliers) are entered once per batch by the
// whole wave, so the scheduler can interleave the independent rows.
// A later scan over tiles and a scatter put the staged outliers in
// block-major order.
#include "dq_device.hpp"
#include "dq_kernels.hpp"

namespace dq {

// Per-lane state of the blocks of one wave step.
template <int DIM, int B, int V>
struct EncState {
    uint32_t rank;  // non-origin outliers found so far in this lane's block
    long long s_all, s_fx, s_fy, s_fz;
    int32_t vmin, vmax;  // block extremes of q (min / max padding)
    uint32_t qo;
    uint32_t dcode[V];
    uint32_t pY[V];
    uint32_t pZ[DIM == 3 ? B : 1][V];

    __device__ __forceinline__ void init() {
        rank = 0;
        s_all = s_fx = s_fy = s_fz = 0;
        vmin = 0x7fffffff;
        vmax = (int32_t)0x80000000;
        qo = 0;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            dcode[j] = 0;
            pY[j] = 0;
        }
#pragma unroll
        for (int k = 0; k < (DIM == 3 ? B : 1); ++k)
#pragma unroll
            for (int j = 0; j < V; ++j) pZ[k][j] = 0;
    }
};

struct WaveCtx {
    uint4* sbuf;
    uint32_t scount;  // LDS staged entries (wave-uniform)
    uint32_t placed;  // entries already in the tile's staging region
    uint32_t t;       // tile
    int lane;
    uint32_t blk0;    // the tile's first block
};

// Dense staging: the slots of block blk in the tile's region (see Staging).
__device__ __forceinline__ uint2* dense_slots(const EncArgs& a, const WaveCtx& w, uint32_t blk) {
    return reinterpret_cast<uint2*>(a.stg.region + (uint64_t)w.t * a.stg.spt) + (uint64_t)(blk - w.blk0) * a.stg.bcells;
}

__device__ __forceinline__ void stage_push(const EncArgs& a, WaveCtx& w, uint32_t tot) {
    if (w.scount + tot > (uint32_t)kStageCap) {
        flush_stage(w.sbuf, w.scount, a.stg, w.t, w.placed, &a.sc->stage_count, w.lane);
        w.scount = 0;
    }
}

__device__ __forceinline__ bool is_inlier(uint32_t u, uint32_t R) { return u - 1u < 2u * R - 1u; }

// Stage the outliers of one row (u = delta + R per cell). Called by the whole
// wave; `origin` marks a lane whose first cell is its block's origin (that
// one is classified at the end of the block).
template <int V>
__device__ __forceinline__ void stage_row_outliers(const EncArgs& a, uint32_t& rank, WaveCtx& w,
                                                   const uint32_t (&u)[V], bool xin, bool origin,
                                                   uint64_t row, uint32_t x0, uint64_t gmask, uint32_t blk) {
    const uint32_t R = (uint32_t)a.R;
    bool out[V];
    uint64_t m[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        out[j] = xin && !is_inlier(u[j], R) && !(j == 0 && origin);
        m[j] = ballot(out[j]);
    }
    uint32_t tot = 0, below = 0, gtot = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        tot += popc(m[j]);
        below += mbcnt(m[j] & gmask);
        gtot += popc(m[j] & gmask);
    }
    if (tot == 0) return;
    if (a.stg.dense) {  // straight to the outlier's own slot
        uint32_t own = 0;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (out[j]) {
                dense_slots(a, w, blk)[1u + rank + below + own] = make_uint2((uint32_t)(row + x0 + j), u[j] - R);
                ++own;
            }
        }
        rank += gtot;
        return;
    }
    stage_push(a, w, tot);
    uint32_t slot = w.scount, own = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        if (out[j]) {
            w.sbuf[slot + mbcnt(m[j])] = make_uint4((uint32_t)(row + x0 + j), u[j] - R, blk, rank + below + own);
            ++own;
        }
        slot += popc(m[j]);
    }
    w.scount = uniform(w.scount + tot);
    rank += gtot;
}

// Pre-quantisation of a batch of rows; the exact path runs once for the
// batch when any lane needs it (see prequant).
template <int V, int NR>
__device__ __forceinline__ void prequant_rows(const float (&xv)[NR][V], double r, double twoeb, double eb,
                                              uint32_t (&q)[NR][V], uint64_t& bad) {
    // x r + 1.5 * 2^52, rounded once, holds the integer nearest to the exact
    // product x r (ties to even) in its low mantissa bits while |x r| < 2^51:
    // its low dword is k mod 2^32, and k = s - 1.5 * 2^52 exactly. The
    // near-half test looks at x r - k (rounded once), as a ballot mask (false
    // for NaN, so a non-finite x fails it); the range test on the running
    // maximum of |k| once for the batch (a product past 2^51 gives |k| past
    // it too).
    uint64_t near = 0;
    double kmax = 0.0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const double xd = (double)xv[i][j];
            const double s = __builtin_fma(xd, r, kRoundShift);
            const double k = s - kRoundShift;
            near |= ballot(!(__builtin_fabs(__builtin_fma(xd, r, -k)) <= kNearHalf));
            kmax = __builtin_fmax(kmax, __builtin_fabs(k));
            q[i][j] = (uint32_t)__builtin_bit_cast(uint64_t, s);
        }
    }
    const bool slow = near != 0 || !(kmax <= kFastMax);
    if (__builtin_expect(ballot(slow) != 0, 0)) {  // slow is wave-uniform except for vmax
        bool out = false;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                double k = __builtin_rint((double)xv[i][j] * r);
                k = exact_round(xv[i][j], k, twoeb, eb);
                const bool ok = __builtin_fabs(k) <= kQMax;  // NaN and +-inf fail too
                out = out || !ok;
                q[i][j] = (uint32_t)(int32_t)(ok ? k : 0.0);
            }
        }
        bad |= ballot(out);
    }
}

// One grid row of a 1-D step (a row of blocks): residuals, codes, statistics,
// outliers.
template <int DIM, int B, int V>
__device__ __forceinline__ void enc_row(const EncArgs& a, EncState<DIM, B, V>& st, WaveCtx& w,
                                        const float (&xv)[V], uint64_t row, uint32_t x0, bool xin, bool leader,
                                        bool last,
                                        uint64_t gmask, uint32_t blk, double r, double twoeb, double eb,
                                        uint64_t& bad) {
    const uint32_t R = (uint32_t)a.R;
    uint32_t q[1][V];
    const float(&x1)[1][V] = reinterpret_cast<const float(&)[1][V]>(xv);
    prequant_rows<V, 1>(x1, r, twoeb, eb, q, bad);
    uint32_t u[V];
    u[0] = q[0][0] - wave_shr1(last ? 0u : q[0][V - 1]) + R;
#pragma unroll
    for (int j = 1; j < V; ++j) u[j] = q[0][j] - q[0][j - 1] + R;
    uint32_t code[V];
    bool anyout = false;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        code[j] = is_inlier(u[j], R) ? u[j] : 0u;
        anyout = anyout || (!is_inlier(u[j], R) && !(j == 0 && leader));
    }
    if (a.pad_mode == PAD_BLOCK) {
        long long rs = 0;
#pragma unroll
        for (int j = 0; j < V; ++j) rs += (int32_t)q[0][j];
        st.s_all += xin ? rs : 0ll;
    } else if (a.pad_mode == PAD_BLOCK_MIN || a.pad_mode == PAD_BLOCK_MAX) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            st.vmin = xin ? min(st.vmin, (int32_t)q[0][j]) : st.vmin;
            st.vmax = xin ? max(st.vmax, (int32_t)q[0][j]) : st.vmax;
        }
    }
    if (leader) {
        st.qo = q[0][0];
#pragma unroll
        for (int j = 0; j < V; ++j) st.dcode[j] = code[j];
    }
    if (xin) store_codes<V>(a.codes + row + x0, code);  // the origin's code is rewritten at block end
    if (ballot(xin && anyout)) stage_row_outliers<V>(a, st.rank, w, u, xin, leader, row, x0, gmask, blk);
}

// A batch of NR consecutive rows (local rows yb .. yb+NR-1 of local plane zl)
// of a 2-D/3-D step. FULL: every row and lane lies inside the field; the
// codes of row i are stored through the tile's buffer resource crs at
// scalar offset csoff + i*nx*2, with no per-lane condition, so every store
// is issued on every path. PB (a pipelined tile past the field's end): the
// same stores, with lanes and rows outside the field sent out of range.
template <int DIM, int B, int V, int NR, bool FULL, bool PB = false>
__device__ __forceinline__ void enc_batch(const EncArgs& a, EncState<DIM, B, V>& st, WaveCtx& w,
                                          const float (&xv)[NR][V], int zl, int yb, uint32_t z, uint32_t y0,
                                          uint32_t x0, bool xin, bool leader, bool last, uint64_t gmask, uint32_t blk,
                                          double r, double twoeb, double eb, uint64_t& bad,
                                          Rsrc crs = Rsrc(), uint32_t csoff = 0) {
    const uint32_t R = (uint32_t)a.R;
    const uint32_t ny = a.g.ny, nx = a.g.nx;
    // phase 1: pre-quantisation of every row
    uint32_t q[NR][V];
    prequant_rows<V, NR>(xv, r, twoeb, eb, q, bad);
    // phase 2: Lorenzo residuals, u = delta + R (rows past the field edge
    // only touch carries no valid row reads)
    uint32_t u[NR][V];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int yl = yb + i;
        // the left neighbour; a block's first lane receives 0 (the zero halo
        // of the x difference) because the last lane of every block sends 0
        uint32_t d[V];
        d[0] = q[i][0] - wave_shr1(last ? 0u : q[i][V - 1]);
#pragma unroll
        for (int j = 1; j < V; ++j) d[j] = q[i][j] - q[i][j - 1];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const uint32_t cur = d[j];
            d[j] = (yl == 0) ? cur : cur - st.pY[j];
            st.pY[j] = cur;
        }
        if constexpr (DIM == 3) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const uint32_t cur = d[j];
                d[j] = cur - st.pZ[yl][j];  // zero on the block's first plane
                st.pZ[yl][j] = cur;
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) u[i][j] = d[j] + R;
    }
    const bool orow0 = (zl == 0) && (yb == 0);  // this batch starts with the block's first row
    // phase 3: codes (the origin's code is rewritten at the end of the block);
    // code 0 marks an outlier, so the smallest code of the batch tells
    // whether the outlier path is needed
    uint32_t cmin = 0xffffffffu;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        uint32_t code[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            code[j] = is_inlier(u[i][j], R) ? u[i][j] : 0u;
            const bool skip = (!FULL && (!xin || y0 + i >= ny)) || (i == 0 && j == 0 && orow0 && leader);
            cmin = min(cmin, skip ? 1u : code[j]);
        }
        if (i == 0 && orow0 && leader) {
            st.qo = q[0][0];
#pragma unroll
            for (int j = 0; j < V; ++j) st.dcode[j] = code[j];
        }
        if constexpr (FULL)
            store_codes_buf<V>(crs, (uint32_t)(w.lane * V * 2), csoff + (uint32_t)i * nx * 2u, code);
        else if constexpr (PB)  // through the tile's resource, lanes and rows outside the field dropped
            store_codes_buf<V>(crs, (xin && y0 + i < ny) ? (uint32_t)(w.lane * V * 2) : kOutOfRange,
                               csoff + (uint32_t)i * nx * 2u, code);
        else if (xin && y0 + i < ny)
            store_codes<V>(a.codes + ((uint64_t)z * ny + y0 + i) * nx + x0, code);
    }
    // padding statistics (Section IV-A: mean, minimum or maximum of the data)
    if (a.pad_mode == PAD_BLOCK || a.pad_mode == PAD_EDGE) {
        const bool pb = a.pad_mode == PAD_BLOCK, pe = !pb;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const bool valid = FULL || (xin && (y0 + i < ny));
            long long rs = 0;
#pragma unroll
            for (int j = 0; j < V; ++j) rs += (int32_t)q[i][j];
            rs = valid ? rs : 0ll;
            st.s_all += pb ? rs : 0ll;
            st.s_fx += (pe && valid && leader) ? (long long)(int32_t)q[i][0] : 0ll;
            st.s_fy += (pe && yb + i == 0) ? rs : 0ll;
            if constexpr (DIM == 3) st.s_fz += (pe && zl == 0) ? rs : 0ll;
        }
    } else if (a.pad_mode == PAD_BLOCK_MIN || a.pad_mode == PAD_BLOCK_MAX) {  // minimum / maximum
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const bool valid = FULL || (xin && (y0 + i < ny));
#pragma unroll
            for (int j = 0; j < V; ++j) {
                st.vmin = valid ? min(st.vmin, (int32_t)q[i][j]) : st.vmin;
                st.vmax = valid ? max(st.vmax, (int32_t)q[i][j]) : st.vmax;
            }
        }
    }
    // phase 4: outliers, rare
    if (ballot(cmin == 0u)) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (!FULL && y0 + i >= ny) continue;  // uniform
            stage_row_outliers<V>(a, st.rank, w, u[i], FULL || xin, i == 0 && orow0 && leader,
                                  ((uint64_t)z * ny + y0 + i) * nx, x0, gmask, blk);
        }
    }
}

// End of the blocks of one wave step: padding values, origin codes and the
// per-block outlier bookkeeping. Returns the step's outlier count.
template <int DIM, int B, int V>
__device__ __forceinline__ uint32_t enc_block_end(const EncArgs& a, EncState<DIM, B, V>& st, WaveCtx& w,
                                                  uint32_t bx, uint32_t by, uint32_t bz, uint32_t blk,
                                                  uint32_t x0, bool gvalid, bool leader, uint32_t gpad,
                                                  uint32_t tile_total) {
    using C = Cfg<DIM, B, V>;
    const uint32_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const uint32_t R = (uint32_t)a.R;
    const int pad = a.pad_mode;
    uint32_t peff = 0;
    if (pad_global(pad)) {
        peff = gpad;
    } else if (pad == PAD_GIVEN) {
        peff = gvalid ? (uint32_t)a.pads[blk] : 0u;
    } else if (pad == PAD_BLOCK_MIN || pad == PAD_BLOCK_MAX) {
        const int32_t P = pad == PAD_BLOCK_MIN ? group_min32<C::GPB>(st.vmin) : group_max32<C::GPB>(st.vmax);
        peff = (uint32_t)P;
        if (leader && gvalid) a.pads[blk] = P;
    } else if (pad != PAD_ZERO) {
        const long long ex = (long long)min((uint32_t)B, nx - min(nx, bx * B));
        const long long ey = DIM >= 2 ? (long long)min((uint32_t)B, ny - by * B) : 1;
        const long long ez = DIM == 3 ? (long long)min((uint32_t)B, nz - bz * B) : 1;
        if (pad == PAD_BLOCK) {
            const long long S = group_sum64<C::GPB>(st.s_all);
            const int32_t P = round_mean(S, gvalid ? ex * ey * ez : 1);
            peff = (uint32_t)P;
            if (leader && gvalid) a.pads[blk] = P;
        } else {
            const long long Sx = group_sum64<C::GPB>(st.s_fx);
            int32_t e[3] = {0, 0, 0};
            if constexpr (DIM == 1) {
                e[0] = (int32_t)st.qo;  // the x face of a 1-D block is its first cell
            } else if constexpr (DIM == 2) {
                const long long Sy = group_sum64<C::GPB>(st.s_fy);
                e[0] = round_mean(Sy, gvalid ? ex : 1);  // axis 0 (y): first row
                e[1] = round_mean(Sx, ey);               // axis 1 (x): first column
            } else {
                const long long Sy = group_sum64<C::GPB>(st.s_fy);
                const long long Sz = group_sum64<C::GPB>(st.s_fz);
                e[0] = round_mean(Sz, gvalid ? ex * ey : 1);  // axis 0 (z): first plane
                e[1] = round_mean(Sy, gvalid ? ex * ez : 1);  // axis 1 (y)
                e[2] = round_mean(Sx, ey * ez);               // axis 2 (x)
            }
            peff = edge_effective<DIM>(e);
            if (leader && gvalid) {
#pragma unroll
                for (int k = 0; k < DIM; ++k) a.pads[(uint64_t)blk * DIM + k] = e[k];
            }
        }
    }
    bool oout = false;
    uint32_t od = 0;
    const uint64_t orow_base = ((uint64_t)(bz * B) * ny + by * B) * nx;
    if (leader && gvalid) {
        od = st.qo - peff;
        const uint32_t u = od + R;
        const bool inl = is_inlier(u, R);
        st.dcode[0] = inl ? u : 0u;
        oout = !inl;
        store_codes<V>(a.codes + orow_base + x0, st.dcode);
    }
    const uint64_t mo = ballot(oout);
    if (mo && a.stg.dense) {
        if (oout) dense_slots(a, w, blk)[0] = make_uint2((uint32_t)(orow_base + x0), od);
    } else if (mo) {
        const uint32_t n = popc(mo);
        stage_push(a, w, n);
        if (oout) w.sbuf[w.scount + mbcnt(mo)] = make_uint4((uint32_t)(orow_base + x0), od, blk, kOriginFlag);
        w.scount = uniform(w.scount + n);
    }
    // per-block outlier counts -> exclusive prefix inside the tile
    const uint32_t cnt = (leader && gvalid) ? st.rank + (oout ? 1u : 0u) : 0u;
    uint32_t excl = 0, step_total = 0;
    if (ballot(cnt != 0)) {
        const uint32_t incl = wave_scan_incl(cnt, w.lane);
        excl = incl - cnt;
        step_total = readlane(incl, 63);
    }
    if (leader && gvalid) a.block_info[blk] = (tile_total + excl) | (oout ? kOriginFlag : 0u);
    return step_total;
}

// The bound of the call a (reduced from the value-range partials by this
// wave) and the call's status so far; the wave that encodes tile 0 reports
// the bound and any bound error.
__device__ __forceinline__ Bound encode_bound(const EncArgs& a, int& st_in, const int lane, const bool first) {
    uint4 pp[kBoundLoads];
    bound_fetch(a.bound, pp, lane);
    st_in = __builtin_nontemporal_load(a.status);  // loaded together with the partials
    const Bound bd = bound_finish(a.bound, pp, lane);
    if (a.bound.nparts && first && lane == 0) {
        *a.eb_out = bd.eb;
        if (bd.status != ST_OK) __hip_atomic_store(a.status, bd.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return bd;
}

// Tile t of the call a, by one wave (sbuf: the wave's LDS staging buffer;
// bd, st_in: from encode_bound).
template <int DIM, int B, int V>
__device__ __forceinline__ void encode_tile(const EncArgs& a, uint4* sbuf, const uint32_t t, const int lane,
                                            const Bound& bd, const int st_in) {
    using C = Cfg<DIM, B, V>;
    WaveCtx w{sbuf, 0u, 0u, t, lane, 0u};
    double r = 0.0, twoeb = 0.0, eb = 0.0;
    uint32_t gpad = 0;
    // false (and the tile's count 0) when the call has already failed
    auto prologue = [&]() -> bool {
        if (bd.status != ST_OK || st_in != ST_OK) {
            if (lane == 0) a.tile_count[t] = 0;
            return false;
        }
        r = bd.r;
        twoeb = bd.twoeb;
        eb = bd.eb;
        if (a.pad_mode == PAD_GLOBAL) {
            gpad = (uint32_t)round_mean((long long)a.sc->sumq, (long long)a.g.N);
            if (t == 0 && lane == 0) a.pads[0] = (int32_t)gpad;
        } else if (a.pad_mode == PAD_GLOBAL_MIN || a.pad_mode == PAD_GLOBAL_MAX) {
            // rounding to the nearest integer is monotone, so the extreme of q
            // is the pre-quantised extreme of x (an out-of-range one fails the
            // call through its own element)
            const float xe = a.pad_mode == PAD_GLOBAL_MIN ? bd.mn : bd.mx;
            const double k = exact_round(xe, __builtin_rint((double)xe * r), twoeb, eb);
            gpad = (uint32_t)(int32_t)(__builtin_fabs(k) <= kQMax ? k : 0.0);
            if (t == 0 && lane == 0) a.pads[0] = (int32_t)gpad;
        }
        return true;
    };
    if (!prologue()) return;
    const uint32_t tx = t % a.g.ntx;
    const uint32_t rr = t / a.g.ntx;
    const uint32_t by = rr % a.g.nby;
    const uint32_t bz = rr / a.g.nby;
    const uint32_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    w.blk0 = (bz * a.g.nby + by) * a.g.nbx + tx * a.g.bpt;

    uint32_t tile_total = 0;  // outliers in this tile so far (wave-uniform)
    uint64_t bad = 0;         // lanes with |q| out of range or x not finite

    if constexpr (!C::WIDE) {
        const int gl = lane & (C::GPB - 1);
        const bool leader = gl == 0;
        const bool last = gl == C::GPB - 1;
        const uint64_t gmask = (C::GPB == 64) ? ~0ull
                                              : (((1ull << C::GPB) - 1) << (lane & ~(C::GPB - 1)));
        if constexpr (DIM == 1) {
            // one row per step: batch NBR steps' loads
            for (int cb = 0; cb < C::XCH; cb += C::NBR) {
                if (tx * C::BPT + cb * C::BPC >= a.g.nbx) break;
                float xv[C::NBR][V];
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const uint32_t x0 = (tx * C::BPT + (cb + i) * C::BPC) * B + (uint32_t)lane * V;
                    load_f<V>(a.x + min(x0, nx - V), xv[i]);  // clamped: always in bounds
                }
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const uint32_t bx0 = tx * C::BPT + (cb + i) * C::BPC;
                    if (bx0 >= a.g.nbx) continue;  // uniform
                    const uint32_t bx = bx0 + (uint32_t)(lane / C::GPB);
                    const bool gvalid = bx < a.g.nbx;
                    const uint32_t x0 = bx0 * B + (uint32_t)lane * V;
                    const bool xin = x0 < nx;
                    EncState<DIM, B, V> st;
                    st.init();
                    enc_row<DIM, B, V>(a, st, w, xv[i], 0, x0, xin, leader, last, gmask, bx, r, twoeb, eb, bad);
                    tile_total += enc_block_end<DIM, B, V>(a, st, w, bx, 0, 0, bx, x0, gvalid, leader,
                                                           gpad, tile_total);
                }
            }
        } else if (C::NBT * C::NBR <= kMaxUnrollRows && (uint64_t)((C::BZ - 1) * ny + C::BY) * nx * 4u < 0x7fffffffull) {
            // Pipelined tile: the block row is one straight-line sequence of
            // NBT batches with kPipeDepth batches of loads in flight ahead of
            // the one being computed, so each wait retires exactly the batch
            // it needs. Interior tiles (FULL: every block complete) load and
            // store unconditionally from wave-uniform row bases. A tile that
            // reaches past the field's end takes the same sequence with the
            // loads clamped to the last column, row and plane (always in
            // bounds), the stores under per-lane conditions and the batches
            // of planes past the end skipped.
            constexpr int NBT = C::NBT;
            constexpr int D = cmin(NBT, kPipeDepth);
            constexpr int YB = C::BY / C::NBR;  // batches per plane
            const uint32_t voff = (uint32_t)lane * V;
            auto run = [&](auto fullI) {
                constexpr bool FULL = decltype(fullI)::value != 0;
                // last local plane and row inside the field
                const uint32_t zmax = FULL ? (uint32_t)C::BZ - 1u : min((uint32_t)C::BZ, nz - bz * C::BZ) - 1u;
                const uint32_t ymax = FULL ? (uint32_t)C::BY - 1u : min((uint32_t)C::BY, ny - by * C::BY) - 1u;
                for (int ch = 0; ch < C::XCH; ++ch) {
                    const uint32_t bx0 = tx * C::BPT + ch * C::BPC;
                    if (!FULL && bx0 >= a.g.nbx) break;  // uniform
                    const uint32_t bx = bx0 + (uint32_t)(lane / C::GPB);
                    const bool gvalid = FULL || bx < a.g.nbx;
                    const uint32_t x0 = bx0 * B + voff;
                    const bool xin = FULL || x0 < nx;
                    // nx is a multiple of V, so a chunk inside the field holds
                    // at least V columns and the clamped offset is >= 0
                    const uint32_t lvoff = FULL ? voff : min(x0, nx - V) - bx0 * B;
                    const uint32_t blk = (bz * a.g.nby + by) * a.g.nbx + bx;
                    const uint64_t base = ((uint64_t)(bz * B) * ny + by * C::BY) * nx + bx0 * B;
                    const Rsrc xrs = make_rsrc(a.x + base);
                    const Rsrc crs = make_rsrc(a.codes + base);
                    EncState<DIM, B, V> st;
                    st.init();
                    float buf[D][C::NBR][V];
                    auto load = [&](auto bI, float (&bb)[C::NBR][V]) {
                        constexpr int b = decltype(bI)::value;
                        const uint32_t zc = FULL ? (uint32_t)(b / YB) : min((uint32_t)(b / YB), zmax);
#pragma unroll
                        for (int i = 0; i < C::NBR; ++i) {
                            const uint32_t yl = (uint32_t)((b % YB) * C::NBR + i);
                            const uint32_t yc = FULL ? yl : min(yl, ymax);
                            load_f_buf<V>(xrs, lvoff * 4u, (zc * ny + yc) * nx * 4u, bb[i]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    };
                    static_for<0, D>([&](auto bI) { load(bI, buf[decltype(bI)::value]); });
                    static_for<0, NBT>([&](auto bI) {
                        constexpr int b = decltype(bI)::value;
                        constexpr int zl = b / YB, yb = (b % YB) * C::NBR;
                        if (FULL || (uint32_t)zl <= zmax)  // uniform
                            enc_batch<DIM, B, V, C::NBR, FULL, !FULL>(a, st, w, buf[b % D], zl, yb, bz * B + zl,
                                                               by * C::BY + yb, x0, xin, leader, last, gmask, blk, r,
                                                               twoeb, eb, bad, crs,
                                                               ((uint32_t)zl * ny + yb) * nx * 2u);
                        if constexpr (b + D < NBT) load(Idx<b + D>{}, buf[b % D]);
                    });
                    tile_total += enc_block_end<DIM, B, V>(a, st, w, bx, by, bz, blk, x0, gvalid, leader, gpad,
                                                           tile_total);
                }
            };
            if ((tx + 1) * C::BPT * B <= nx && (by + 1) * C::BY <= ny && (bz + 1) * C::BZ <= nz)
                run(Idx<1>{});
            else
                run(Idx<0>{});
        } else {
            for (int ch = 0; ch < C::XCH; ++ch) {
                const uint32_t bx0 = tx * C::BPT + ch * C::BPC;
                if (bx0 >= a.g.nbx) break;
                const uint32_t bx = bx0 + (uint32_t)(lane / C::GPB);
                const bool gvalid = bx < a.g.nbx;
                const uint32_t x0 = bx0 * B + (uint32_t)lane * V;
                const bool xin = x0 < nx;
                const uint32_t xl = min(x0, nx - V);  // clamped load column
                const uint32_t blk = (bz * a.g.nby + by) * a.g.nbx + bx;
                EncState<DIM, B, V> st;
                st.init();
                // batches of NBR rows in local row-major order; the next batch
                // is loaded while the current one is computed
                constexpr int YB = C::BY / C::NBR;  // batches per plane
                auto load_batch = [&](int zl, int yb, float (&buf)[C::NBR][V]) {
                    const uint32_t z = bz * B + zl;
#pragma unroll
                    for (int i = 0; i < C::NBR; ++i) {
                        const uint32_t y = min(by * B + yb + i, ny - 1);  // clamped row
                        load_f<V>(a.x + ((uint64_t)z * ny + y) * nx + xl, buf[i]);
                    }
                    // keep the loads here: the scheduler would otherwise sink
                    // them to their first use and serialise memory and compute
                    __builtin_amdgcn_sched_barrier(0);
                };
                auto compute_batch = [&](int zl, int yb, float (&buf)[C::NBR][V]) {
                    enc_batch<DIM, B, V, C::NBR, false>(a, st, w, buf, zl, yb, bz * B + zl, by * B + yb, x0, xin,
                                                 leader, last, gmask, blk, r, twoeb, eb, bad);
                };
                float bufA[C::NBR][V], bufB[C::NBR][V];
                if constexpr (DIM == 3 && YB == 2) {
                    // two batches per plane: buffer A holds rows 0..NBR-1, B the rest
                    const int nzl = (int)min((uint32_t)B, nz - bz * B);
                    load_batch(0, 0, bufA);
                    for (int zl = 0; zl < nzl; ++zl) {
                        load_batch(zl, C::NBR, bufB);
                        compute_batch(zl, 0, bufA);
                        if (zl + 1 < nzl) load_batch(zl + 1, 0, bufA);
                        compute_batch(zl, C::NBR, bufB);
                    }
                } else {
                    static_assert(DIM == 2 || YB == 1, "3-D batches cover a whole plane or half of it");
                    // batch b covers plane b / YB, rows (b % YB) * NBR ...
                    const int nbt = DIM == 3 ? (int)min((uint32_t)B, nz - bz * B)
                                             : (int)((min((uint32_t)B, ny - by * B) + C::NBR - 1) / C::NBR);
                    load_batch(0, 0, bufA);
                    // both buffers in flight, issued in the order they are
                    // consumed, so each wait covers only the batch it needs
                    if (nbt > 1) load_batch(1 / YB, (1 % YB) * C::NBR, bufB);
                    for (int b = 0; b < nbt; b += 2) {
                        compute_batch(b / YB, (b % YB) * C::NBR, bufA);
                        if (b + 2 < nbt) load_batch((b + 2) / YB, ((b + 2) % YB) * C::NBR, bufA);
                        if (b + 1 < nbt) {
                            compute_batch((b + 1) / YB, ((b + 1) % YB) * C::NBR, bufB);
                            if (b + 3 < nbt) load_batch((b + 3) / YB, ((b + 3) % YB) * C::NBR, bufB);
                        }
                    }
                }
                tile_total += enc_block_end<DIM, B, V>(a, st, w, bx, by, bz, blk, x0, gvalid, leader, gpad,
                                                       tile_total);
            }
        }
    } else {
        // 1-D blocks wider than one wave step: blocks one after another
        const uint32_t R = (uint32_t)a.R;
        for (int bi = 0; bi < C::BPT; ++bi) {
            const uint32_t bx = tx * C::BPT + bi;
            if (bx >= a.g.nbx) break;
            uint32_t rank = 0, carry = 0, qo = 0;
            long long s_all = 0;
            int32_t vmin = 0x7fffffff, vmax = (int32_t)0x80000000;
            uint32_t dcode[V];
#pragma unroll
            for (int j = 0; j < V; ++j) dcode[j] = 0;
            for (int cb = 0; cb < C::NCH; cb += C::NBR) {
                if (bx * B + cb * C::CX >= nx) break;
                float xv[C::NBR][V];
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const uint32_t x0 = bx * B + (cb + i) * C::CX + (uint32_t)lane * V;
                    load_f<V>(a.x + min(x0, nx - V), xv[i]);
                }
                uint32_t q[C::NBR][V];
                prequant_rows<V, C::NBR>(xv, r, twoeb, eb, q, bad);
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const int ch = cb + i;
                    const uint32_t xc = bx * B + ch * C::CX;
                    if (xc >= nx) continue;  // uniform
                    const uint32_t x0 = xc + (uint32_t)lane * V;
                    const bool xin = x0 < nx;
                    uint32_t left = wave_shr1(q[i][V - 1]);
                    if (lane == 0) left = carry;  // 0 at the block start
                    carry = readlane(q[i][V - 1], 63);
                    uint32_t u[V];
                    u[0] = q[i][0] - left + R;
#pragma unroll
                    for (int j = 1; j < V; ++j) u[j] = q[i][j] - q[i][j - 1] + R;
                    const bool origin_lane = (ch == 0) && (lane == 0);
                    uint32_t code[V];
                    bool anyout = false;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        code[j] = is_inlier(u[j], R) ? u[j] : 0u;
                        anyout = anyout || (!is_inlier(u[j], R) && !(j == 0 && origin_lane));
                    }
                    if (a.pad_mode == PAD_BLOCK && xin) {
#pragma unroll
                        for (int j = 0; j < V; ++j) s_all += (int32_t)q[i][j];
                    } else if ((a.pad_mode == PAD_BLOCK_MIN || a.pad_mode == PAD_BLOCK_MAX) && xin) {
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            vmin = min(vmin, (int32_t)q[i][j]);
                            vmax = max(vmax, (int32_t)q[i][j]);
                        }
                    }
                    if (origin_lane) {
                        qo = q[i][0];
#pragma unroll
                        for (int j = 0; j < V; ++j) dcode[j] = code[j];
                    }
                    if (xin) store_codes<V>(a.codes + x0, code);  // origin rewritten at block end
                    if (ballot(xin && anyout))
                        stage_row_outliers<V>(a, rank, w, u, xin, origin_lane, 0, x0, ~0ull, bx);
                }
            }
            uint32_t peff = 0;
            if (pad_global(a.pad_mode)) {
                peff = gpad;
            } else if (a.pad_mode == PAD_GIVEN) {
                peff = (uint32_t)a.pads[bx];
            } else if (a.pad_mode == PAD_BLOCK_MIN || a.pad_mode == PAD_BLOCK_MAX) {
                const int32_t P = a.pad_mode == PAD_BLOCK_MIN ? group_min32<64>(vmin) : group_max32<64>(vmax);
                peff = (uint32_t)P;
                if (lane == 0) a.pads[bx] = P;
            } else if (a.pad_mode == PAD_BLOCK) {
                const long long S = group_sum64<64>(s_all);
                const long long ex = (long long)min((uint32_t)B, nx - bx * B);
                const int32_t P = round_mean(S, ex);
                peff = (uint32_t)P;
                if (lane == 0) a.pads[bx] = P;
            } else if (a.pad_mode == PAD_EDGE) {
                peff = readlane(qo, 0);
                if (lane == 0) a.pads[bx] = (int32_t)peff;
            }
            bool oout = false;
            uint32_t od = 0;
            if (lane == 0) {
                od = qo - peff;
                const uint32_t u = od + R;
                const bool inl = is_inlier(u, R);
                dcode[0] = inl ? u : 0u;
                oout = !inl;
                store_codes<V>(a.codes + (uint64_t)bx * B, dcode);
            }
            if (ballot(oout) && a.stg.dense) {
                if (lane == 0) dense_slots(a, w, bx)[0] = make_uint2(bx * B, od);
            } else if (ballot(oout)) {
                stage_push(a, w, 1);
                if (lane == 0) w.sbuf[w.scount] = make_uint4(bx * B, od, bx, kOriginFlag);
                w.scount = uniform(w.scount + 1);
            }
            const uint32_t cnt = readlane(rank + (oout ? 1u : 0u), 0);
            if (lane == 0) a.block_info[bx] = tile_total | (oout ? kOriginFlag : 0u);
            tile_total += cnt;
        }
    }

    if (w.scount) flush_stage(w.sbuf, w.scount, a.stg, t, w.placed, &a.sc->stage_count, lane);
    if (lane == 0) a.tile_count[t] = tile_total;
    if (bad && lane == 0) __hip_atomic_store(a.status, ST_ERANGE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One value per lane (V = 1) gives twice the tiles of V = 2; the register
// budget is capped so that four waves fit on every SIMD.
template <int DIM, int B, int V>
__global__ __launch_bounds__(kThreads, (V == 1 ? 4 : 1)) void k_encode(EncArgs a) {
    __shared__ uint4 sbuf_all[kWaves][kStageCap];
    const int wave = (int)uniform(threadIdx.x >> 6);  // scalar: tile math stays in SGPRs
    const int lane = threadIdx.x & 63;
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x) * kWaves + wave;
    if (t >= a.g.n_tiles) return;
    int st_in = 0;
    const Bound bd = encode_bound(a, st_in, lane, t == 0);
    encode_tile<DIM, B, V>(a, sbuf_all[wave], t, lane, bd, st_in);
}

// Persistent encode of a batch of fields of one configuration: every
// workgroup takes the next unit of the flattened (field, run of tiles) queue
// with an atomic ticket until the queue is drained (all waves of a workgroup
// see the same ticket, so all reach the exit test together); its waves
// encode the unit's tiles in turn, wave w the tiles t0 + w, t0 + w + 4, ...,
// so the four waves work on adjacent tiles at a time, as in the per-call
// kernel. The tables are restrict-qualified read-only kernel parameters, so
// the compiler may load a field's arguments with scalar loads (and load them
// again) instead of keeping them in vector registers; each wave reduces the
// field's bound once per unit.
template <int DIM, int B, int V>
__global__ __launch_bounds__(kThreads, (V == 1 ? 4 : 1)) void k_encode_batch(const EncArgs* __restrict__ enc,
                                                                             const uint4* __restrict__ units,
                                                                             uint32_t n_units,
                                                                             unsigned int* ticket) {
    __shared__ uint4 sbuf_all[kWaves][kStageCap];
    __shared__ uint32_t s_unit;
    const int wave = (int)uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (;;) {
        if (threadIdx.x == 0) s_unit = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t u = uniform(s_unit);
        __syncthreads();  // read by every wave before the next ticket replaces it
        if (u >= n_units) break;
        const uint4 un = units[u];  // field, first tile, tiles
        const EncArgs& a = enc[uniform(un.x)];
        const uint32_t t0 = uniform(un.y), t1 = t0 + uniform(un.z);
        if (t0 + (uint32_t)wave >= t1) continue;
        int st_in = 0;
        const Bound bd = encode_bound(a, st_in, lane, t0 + (uint32_t)wave == 0);
        for (uint32_t t = t0 + (uint32_t)wave; t < t1; t += kWaves)
            encode_tile<DIM, B, V>(a, sbuf_all[wave], t, lane, bd, st_in);
    }
}

#ifndef DQ_DIM
#error "dq_encode.hip is compiled once per DQ_DIM (1, 2, 3)"
#endif

// instantiated only for the configurations of this object's dimensionality
template <int D, int BB, int VV>
static bool try_launch_encode(int block, int v, const EncArgs& a, dim3 grid, hipStream_t stream) {
    if constexpr (D == DQ_DIM) {
        if (block == BB && v == VV) {
            hipLaunchKernelGGL((k_encode<D, BB, VV>), grid, dim3(kThreads), 0, stream, a);
            return true;
        }
    }
    return false;
}

#define DQ_ENC_CASE(D, BB, VV) \
    if (try_launch_encode<D, BB, VV>(block, v, a, grid, stream)) return true;

bool DQ_CAT(launch_encode_dim, DQ_DIM)(int block, int v, const EncArgs& a, dim3 grid, hipStream_t stream) {
    DQ_CONFIGS(DQ_ENC_CASE)
    return false;
}

template <int D, int BB, int VV>
static bool try_launch_encode_batch(int block, int v, const BatchQueue& q, int grid, hipStream_t stream) {
    if constexpr (D == DQ_DIM) {
        if (block == BB && v == VV) {
            int per_cu = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(
                    &k_encode_batch<D, BB, VV>), kThreads, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            const int resident = per_cu * cus;
            hipLaunchKernelGGL((k_encode_batch<D, BB, VV>), dim3((uint32_t)(grid < resident ? grid : resident)),
                               dim3(kThreads), 0, stream, q.enc, q.units, q.n_units, q.ticket);
            return true;
        }
    }
    return false;
}

#define DQ_ENCB_CASE(D, BB, VV) \
    if (try_launch_encode_batch<D, BB, VV>(block, v, q, grid, stream)) return true;

bool DQ_CAT(launch_encode_batch_dim, DQ_DIM)(int block, int v, const BatchQueue& q, int grid, hipStream_t stream) {
    DQ_CONFIGS(DQ_ENCB_CASE)
    return false;
}

template <int D, int BB, int VV>
static int try_encode_occupancy(int block, int v) {
    if constexpr (D == DQ_DIM) {
        if (block == BB && v == VV) {
            int n = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_encode<D, BB, VV>),
                                                             kThreads, 0) != hipSuccess)
                return 0;
            return n;
        }
    }
    return -1;
}

#define DQ_OCC_CASE(D, BB, VV)                                          \
    {                                                                   \
        const int n = try_encode_occupancy<D, BB, VV>(block, v);        \
        if (n >= 0) return n;                                           \
    }

int DQ_CAT(encode_occupancy_dim, DQ_DIM)(int block, int v) {
    DQ_CONFIGS(DQ_OCC_CASE)
    return 0;
}

}  // namespace dq
