// dq_decode.hip - fused dual-quantisation decode kernel (gfx950).
//
// Decompression reverses the prediction (Section III-A). The residual of the
// zero-padded Lorenzo predictor is the mixed backward difference along every
// axis, so its inverse inside a block is the n-D inclusive prefix sum; the
// padding enters only through the block origin, so
//     q(u) = P_eff + sum_{w <= u, same block} delta(w).
// Per tile: load a batch of rows of uint16 codes (V per lane, all loads in
// flight before the first use); delta = code - R, or the outlier value looked
// up by its rank inside the block; in-lane prefix over the V cells, segmented
// DPP scan over the GPB lanes of each block row, running sums over rows (y)
// and planes (z) in registers, add P_eff, and dequantise
// x_hat = (float)((double)q * 2eb) with one fp64 product.
#include "dq_device.hpp"
#include "dq_kernels.hpp"

namespace dq {

template <int DIM>
__device__ __forceinline__ uint32_t block_peff(const DecArgs& a, uint32_t blk) {
    const int pad = a.pad_mode;
    if (pad == PAD_ZERO) return 0u;
    if (pad_global(pad)) return (uint32_t)a.pads[0];
    if (pad_per_block(pad)) return (uint32_t)a.pads[blk];
    int32_t e[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) e[k] = a.pads[(uint64_t)blk * DIM + k];
    return edge_effective<DIM>(e);
}

// The first outliers of a wave's run of blocks, one per lane (idx, val of
// entry base + lane for lane < cnt): zero codes take their outlier from here
// with a lane shuffle instead of a load issued behind the prefetched codes.
struct OutWin {
    uint32_t idx = 0, val = 0;
    uint32_t base = 0, cnt = 0;  // wave-uniform
};

template <int DIM, int B, int V>
struct DecState {
    uint32_t rank;  // zero codes seen so far in this lane's block
    uint32_t os, oe;  // outlier run of the block
    OutWin win;
    uint32_t peff;
    uint32_t pY[V];
    uint32_t pZ[DIM == 3 ? B : 1][V];

    __device__ __forceinline__ void init(const DecArgs& a, uint32_t blk, bool gvalid) {
        rank = 0;
        os = oe = 0;
        if (a.n_out && gvalid) block_run(a, blk, os, oe);
        peff = gvalid ? block_peff<DIM>(a, blk) : 0u;
#pragma unroll
        for (int j = 0; j < V; ++j) pY[j] = 0;
#pragma unroll
        for (int k = 0; k < (DIM == 3 ? B : 1); ++k)
#pragma unroll
            for (int j = 0; j < V; ++j) pZ[k][j] = 0;
    }

    // Load the window; lanes 0 .. last hold valid blocks in lane order (lane
    // last in the wave's last valid block), so the wave's outliers are
    // entries os(lane 0) .. oe(lane last). Block starts lie in [0, n_out] but
    // need not increase over a list out of order (whose call ends in
    // ECORRUPT): an empty window then, never a wrapped count.
    __device__ __forceinline__ void prefetch(const DecArgs& a, int lane, int last = 63) {
        win.base = uniform(os);
        const uint32_t e63 = readlane(oe, last);
        win.cnt = e63 > win.base ? min(e63 - win.base, 64u) : 0u;
        if (win.cnt) {
            const uint32_t k = win.base + min((uint32_t)lane, win.cnt - 1u);
            win.idx = a.out_idx[k];
            win.val = (uint32_t)a.out_val[k];
        }
    }
};

// Replace zero codes of this row by their outliers: the k-th zero code of a
// block (local row-major order) is the block's k-th outlier.
template <int V>
__device__ __forceinline__ void fetch_outliers(const DecArgs& a, const uint32_t (&c)[V], uint32_t (&d)[V],
                                               uint32_t& rank, uint32_t os, uint32_t oe, uint64_t gmask,
                                               uint64_t gbase, bool& corrupt, const OutWin& w = OutWin{}) {
    bool anyzero = false;
#pragma unroll
    for (int j = 0; j < V; ++j) anyzero = anyzero || c[j] == 0u;
    if (ballot(anyzero)) {  // rare: entered by the whole wave
        uint64_t m[V];
#pragma unroll
        for (int j = 0; j < V; ++j) m[j] = ballot(c[j] == 0u);
        uint32_t below = 0, gtot = 0, own = 0;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            below += mbcnt(m[j] & gmask);
            gtot += popc(m[j] & gmask);
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const bool z = c[j] == 0u;
            const uint32_t k = os + rank + below + own;
            own += z ? 1u : 0u;
            const uint32_t kk = k - w.base;
            uint32_t wi = 0, wv = 0;
            if (w.cnt) {  // uniform: every lane takes part in the shuffle
                const int src = (int)min(kk, 63u);
                wi = (uint32_t)__shfl((int)w.idx, src);
                wv = (uint32_t)__shfl((int)w.val, src);
            }
            if (z) {
                bool have = false;
                if (k < oe) {
                    have = true;
                    if (kk >= w.cnt) {
                        wi = a.out_idx[k];
                        wv = (uint32_t)a.out_val[k];
                    }
                }
                if (have && wi == (uint32_t)(gbase + j)) {
                    d[j] = wv;
                } else {
                    corrupt = true;
                    d[j] = 0;
                }
            }
        }
        rank += gtot;
    }
}

// The same for every row of a batch at once. A row's entry indices follow
// from the codes alone, so the loads of all entries past the window are
// issued before any is used: the batch waits once for them instead of once
// per row (each wait also covers the code loads prefetched behind it).
template <int V, int NR, bool FULL>
__device__ __forceinline__ void fetch_outliers_batch(const DecArgs& a, const uint32_t (&c)[NR][V],
                                                     uint32_t (&d)[NR][V], uint32_t& rank, uint32_t os, uint32_t oe,
                                                     uint64_t gmask, uint64_t gbase, uint64_t row_stride, bool xin,
                                                     uint32_t y0, bool& corrupt, const OutWin& w) {
    uint32_t wi[NR][V], wv[NR][V];
    bool zero[NR][V], have[NR][V];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const bool rowin = FULL || y0 + (uint32_t)i < a.g.ny;  // uniform
        uint64_t m[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            zero[i][j] = rowin && (FULL || xin) && c[i][j] == 0u;
            m[j] = ballot(zero[i][j]);
        }
        uint32_t below = 0, gtot = 0, own = 0;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            below += mbcnt(m[j] & gmask);
            gtot += popc(m[j] & gmask);
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const uint32_t k = os + rank + below + own;
            own += zero[i][j] ? 1u : 0u;
            const uint32_t kk = k - w.base;
            uint32_t ei = 0, ev = 0;
            if (w.cnt) {  // uniform: every lane takes part in the shuffle
                const int src = (int)min(kk, 63u);
                ei = (uint32_t)__shfl((int)w.idx, src);
                ev = (uint32_t)__shfl((int)w.val, src);
            }
            have[i][j] = zero[i][j] && k < oe;
            if (have[i][j] && kk >= w.cnt) {
                ei = a.out_idx[k];
                ev = (uint32_t)a.out_val[k];
            }
            wi[i][j] = ei;
            wv[i][j] = ev;
        }
        rank += gtot;
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (zero[i][j]) {
                if (have[i][j] && wi[i][j] == (uint32_t)(gbase + (uint64_t)i * row_stride + (uint64_t)j)) {
                    d[i][j] = wv[i][j];
                } else {
                    corrupt = true;
                    d[i][j] = 0;
                }
            }
        }
    }
}

template <int DIM, int B, int V>
__device__ __forceinline__ void dec_row(const DecArgs& a, DecState<DIM, B, V>& st, const uint32_t (&c)[V], int yl,
                                        uint64_t row, uint32_t x0, bool xin, uint64_t gmask, int lane,
                                        bool& corrupt) {
    using C = Cfg<DIM, B, V>;
    const uint32_t R = (uint32_t)a.R;
    uint32_t cc[V], d[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        cc[j] = xin ? c[j] : R;  // lanes past the field edge decode zeros
        d[j] = cc[j] - R;
    }
    fetch_outliers<V>(a, cc, d, st.rank, st.os, st.oe, gmask, row + x0, corrupt);
    // x: in-lane prefix, then segmented scan across the block row
    uint32_t s[V];
    s[0] = d[0];
#pragma unroll
    for (int j = 1; j < V; ++j) s[j] = s[j - 1] + d[j];
    const uint32_t incl = seg_scan_incl<C::GPB>(s[V - 1], lane);
    const uint32_t excl = incl - s[V - 1];
    float o[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        uint32_t p = s[j] + excl;
        if constexpr (DIM >= 2) {
            p = (yl == 0) ? p : p + st.pY[j];
            st.pY[j] = p;
        }
        if constexpr (DIM == 3) {
            p = p + st.pZ[yl][j];  // zero on the block's first plane
            st.pZ[yl][j] = p;
        }
        const int32_t q = (int32_t)(p + st.peff);
        o[j] = (float)((double)q * a.twoeb);
    }
    if (xin) store_f<V>(a.x_hat + row + x0, o);
}

// A batch of NR consecutive rows (local rows yb .. yb+NR-1 of local plane zl)
// of a 2-D/3-D step: the outlier lookup is entered once per batch by the
// whole wave, the prefix sums and dequantisation are branch-free across rows.
// FULL: every row and lane lies inside the field; row i is written through
// the tile's buffer resource ors at scalar offset osoff + i*nx*4, with no
// per-lane condition. PB (a pipelined tile past the field's end): the same
// stores, with lanes and rows outside the field sent out of range.
template <int DIM, int B, int V, int NR, bool FULL, bool PB = false, bool SPLIT = false>
__device__ __forceinline__ void dec_batch(const DecArgs& a, DecState<DIM, B, V>& st, const uint32_t (&c)[NR][V],
                                          int yb, uint32_t z, uint32_t y0, uint32_t x0, bool xin, uint64_t gmask,
                                          int lane, bool& corrupt, Rsrc ors = Rsrc(), uint32_t osoff = 0,
                                          uint32_t obase = 0) {
    using C = Cfg<DIM, B, V>;
    const uint32_t R = (uint32_t)a.R;
    const uint32_t ny = a.g.ny, nx = a.g.nx;
    uint32_t d[NR][V];
    bool anyzero = false;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const uint32_t cc = (FULL || xin) ? c[i][j] : R;  // lanes past the field edge decode zeros
            d[i][j] = cc - R;
            anyzero = anyzero || (cc == 0u && (FULL || y0 + i < ny));
        }
    }
    if (ballot(anyzero)) {  // rare: rows in order, so ranks follow local row-major order
        if constexpr (NR * V <= 4) {
            // small batches (the small blocks that outlier-dense fields tune
            // to): one wait for the whole batch's entries
            fetch_outliers_batch<V, NR, FULL>(a, c, d, st.rank, st.os, st.oe, gmask,
                                              ((uint64_t)z * ny + y0) * nx + x0, nx, xin, y0, corrupt, st.win);
        } else {
            // larger batches row by row: holding every row's entries would
            // cost the kernel occupancy on every field, outliers or not
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                if (!FULL && y0 + i >= ny) continue;  // uniform
                uint32_t cc[V];
#pragma unroll
                for (int j = 0; j < V; ++j) cc[j] = (FULL || xin) ? c[i][j] : R;
                fetch_outliers<V>(a, cc, d[i], st.rank, st.os, st.oe, gmask,
                                  ((uint64_t)z * ny + y0 + i) * nx + x0, corrupt, st.win);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int yl = yb + i;
        // x: in-lane prefix, then segmented scan across the block row
        uint32_t s[V];
        s[0] = d[i][0];
#pragma unroll
        for (int j = 1; j < V; ++j) s[j] = s[j - 1] + d[i][j];
        const uint32_t incl = seg_scan_incl<C::GPB>(s[V - 1], lane);
        const uint32_t excl = incl - s[V - 1];
        float o[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            uint32_t p = s[j] + excl;
            p = (yl == 0) ? p : p + st.pY[j];
            st.pY[j] = p;
            if constexpr (DIM == 3) {
                p = p + st.pZ[yl][j];  // zero on the block's first plane
                st.pZ[yl][j] = p;
            }
            const int32_t q = (int32_t)(p + st.peff);
            o[j] = (float)((double)q * a.twoeb);
        }
        if constexpr ((FULL || PB) && SPLIT) {
            // two unconditional stores, each lane in one of them: nontemporal for
            // lanes on whole lines of the segment, write-back for lanes on lines
            // shared with the neighbouring segment (so the two parts merge in the
            // L2), the other store of the pair out of range
            const uint32_t soff = osoff + (uint32_t)i * nx * 4u;
            const uint32_t lof = (uint32_t)(lane * V * 4);
            const uint32_t xs = x0 - (uint32_t)lane * V;  // the segment's first column
            const uint32_t lo = obase + soff;
            const uint32_t hi = lo + (FULL ? 256u * V : (min(xs + 64u * V, nx) - xs) * 4u);
            const bool valid = FULL || (xin && y0 + i < ny);
            const bool sh = shares_line(lo + lof, lo, hi);
            store_f_buf<V>(ors, (valid && !sh) ? lof : kOutOfRange, soff, o);
            store_f_buf<V, kPolDefault>(ors, (valid && sh) ? lof : kOutOfRange, soff, o);
        } else if constexpr (FULL) {
            store_f_buf<V>(ors, (uint32_t)(lane * V * 4), osoff + (uint32_t)i * nx * 4u, o);
        } else if constexpr (PB) {  // through the tile's resource, lanes and rows outside the field dropped
            store_f_buf<V>(ors, (xin && y0 + i < ny) ? (uint32_t)(lane * V * 4) : kOutOfRange,
                           osoff + (uint32_t)i * nx * 4u, o);
        } else if (xin && y0 + i < ny) {
            store_f<V>(a.x_hat + ((uint64_t)z * ny + y0 + i) * nx + x0, o);
        }
    }
}


// Tile t of the call a, by one wave (NTC: nontemporal code loads; SPLIT:
// decoded rows stored as a nontemporal / write-back pair, see dec_batch).
template <int DIM, int B, int V, bool NTC = false, bool SPLIT = false>
__device__ __forceinline__ void decode_tile(DecArgs a, const uint32_t t, const int lane) {
    using C = Cfg<DIM, B, V>;
    if (a.src) {  // the outlier count and bound of the compress call that wrote this stream
        const int sst = (int)uniform((uint32_t)a.src->status);
        const unsigned long long n = a.src->n_out;
        a.eb_abs = uniform(a.src->eb_abs);
        a.twoeb = 2.0 * a.eb_abs;
        a.n_out = uniform((uint32_t)(n < a.cap ? n : a.cap));
        if (sst != ST_OK) {  // nothing valid to decode: pass the compress status on
            if (t == 0 && lane == 0) {
                *a.n_out_out = n;
                *a.eb_out = a.eb_abs;
                status_set_tagged(a.res_word, a.tag, sst);
            }
            return;
        }
    }
    if (t == 0 && lane == 0) {  // the call's result (status: see status_init_tagged)
        *a.n_out_out = a.n_out;
        *a.eb_out = a.eb_abs;
        status_init_tagged(a.res_word, a.tag);
    }
    const uint32_t tx = t % a.g.ntx;
    const uint32_t rr = t / a.g.ntx;
    const uint32_t by = rr % a.g.nby;
    const uint32_t bz = rr / a.g.nby;
    const uint32_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    bool corrupt = false;

    if constexpr (!C::WIDE) {
        const int gl = lane & (C::GPB - 1);
        const bool leader = gl == 0;
        const uint64_t gmask = (C::GPB == 64) ? ~0ull
                                              : (((1ull << C::GPB) - 1) << (lane & ~(C::GPB - 1)));
        if constexpr (DIM == 1) {
            for (int cb = 0; cb < C::XCH; cb += C::NBR) {
                if (tx * C::BPT + cb * C::BPC >= a.g.nbx) break;
                uint32_t c[C::NBR][V];
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const uint32_t x0 = (tx * C::BPT + (cb + i) * C::BPC) * B + (uint32_t)lane * V;
                    load_codes<V, NTC>(a.codes + min(x0, nx - V), c[i]);  // clamped: always in bounds
                }
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const uint32_t bx0 = tx * C::BPT + (cb + i) * C::BPC;
                    if (bx0 >= a.g.nbx) continue;  // uniform
                    const uint32_t bx = bx0 + (uint32_t)(lane / C::GPB);
                    const bool gvalid = bx < a.g.nbx;
                    const uint32_t x0 = bx0 * B + (uint32_t)lane * V;
                    DecState<DIM, B, V> st;
                    st.init(a, bx, gvalid);
                    dec_row<DIM, B, V>(a, st, c[i], 0, 0, x0, x0 < nx, gmask, lane, corrupt);
                    if (leader && gvalid && st.rank != st.oe - st.os) corrupt = true;
                }
            }
        } else if (C::NBT * C::NBR <= kMaxUnrollRows && (uint64_t)((C::BZ - 1) * ny + C::BY) * nx * 4u < 0x7fffffffull) {
            // Pipelined tile: the block row is one straight-line sequence of
            // NBT batches with kPipeDepth batches of loads in flight ahead of
            // the one being decoded. Interior tiles (FULL) load and store
            // unconditionally from wave-uniform row bases; a tile that reaches
            // past the field's end loads clamped columns, rows and planes
            // (always in bounds), stores under per-lane conditions and skips
            // the batches of planes past the end.
            constexpr int NBT = C::NBT;
            constexpr int D = cmin(NBT, kPipeDepth);
            constexpr int YB = C::BY / C::NBR;  // batches per plane
            const uint32_t voff = (uint32_t)lane * V;
            auto run = [&](auto fullI) {
                constexpr bool FULL = decltype(fullI)::value != 0;
                const uint32_t zmax = FULL ? (uint32_t)C::BZ - 1u : min((uint32_t)C::BZ, nz - bz * C::BZ) - 1u;
                const uint32_t ymax = FULL ? (uint32_t)C::BY - 1u : min((uint32_t)C::BY, ny - by * C::BY) - 1u;
                for (int ch = 0; ch < C::XCH; ++ch) {
                    const uint32_t bx0 = tx * C::BPT + ch * C::BPC;
                    if (!FULL && bx0 >= a.g.nbx) break;  // uniform
                    const uint32_t bx = bx0 + (uint32_t)(lane / C::GPB);
                    const bool gvalid = FULL || bx < a.g.nbx;
                    const uint32_t x0 = bx0 * B + voff;
                    const bool xin = FULL || x0 < nx;
                    // nx is a multiple of V: the clamped offset is >= 0
                    const uint32_t lvoff = FULL ? voff : min(x0, nx - V) - bx0 * B;
                    const uint32_t blk = (bz * a.g.nby + by) * a.g.nbx + bx;
                    const uint64_t base = ((uint64_t)(bz * B) * ny + by * C::BY) * nx + bx0 * B;
                    const Rsrc crs = make_rsrc(a.codes + base);
                    const Rsrc ors = make_rsrc(a.x_hat + base);
                    const uint32_t obase = (uint32_t)reinterpret_cast<uintptr_t>(a.x_hat + base);
                    DecState<DIM, B, V> st;
                    st.init(a, blk, gvalid);
                    uint32_t buf[D][C::NBR][V];
                    auto load = [&](auto bI, uint32_t (&bb)[C::NBR][V]) {
                        constexpr int b = decltype(bI)::value;
                        const uint32_t zc = FULL ? (uint32_t)(b / YB) : min((uint32_t)(b / YB), zmax);
#pragma unroll
                        for (int i = 0; i < C::NBR; ++i) {
                            const uint32_t yl = (uint32_t)((b % YB) * C::NBR + i);
                            const uint32_t yc = FULL ? yl : min(yl, ymax);
                            load_codes_buf<V, NTC>(crs, lvoff * 2u, (zc * ny + yc) * nx * 2u, bb[i]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    };
                    static_for<0, D>([&](auto bI) { load(bI, buf[decltype(bI)::value]); });
                    if (a.n_out) {
                        // the last lane of the chunk's last block inside the field
                        const uint32_t nvb = FULL ? (uint32_t)C::BPC : min((uint32_t)C::BPC, a.g.nbx - bx0);
                        st.prefetch(a, lane, (int)(nvb * C::GPB) - 1);
                    }
                    static_for<0, NBT>([&](auto bI) {
                        constexpr int b = decltype(bI)::value;
                        constexpr int zl = b / YB, yb = (b % YB) * C::NBR;
                        if (FULL || (uint32_t)zl <= zmax)  // uniform
                            dec_batch<DIM, B, V, C::NBR, FULL, !FULL, SPLIT>(
                                a, st, buf[b % D], yb, bz * B + zl, by * C::BY + yb, x0, xin, gmask, lane, corrupt,
                                ors, ((uint32_t)zl * ny + yb) * nx * 4u, obase);
                        if constexpr (b + D < NBT) load(Idx<b + D>{}, buf[b % D]);
                    });
                    if (leader && gvalid && st.rank != st.oe - st.os) corrupt = true;
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
                const uint32_t xl = min(x0, nx - V);
                const uint32_t blk = (bz * a.g.nby + by) * a.g.nbx + bx;
                DecState<DIM, B, V> st;
                st.init(a, blk, gvalid);
                // batches of NBR rows; the next batch is loaded while the
                // current one is decoded
                constexpr int YB = C::BY / C::NBR;  // batches per plane
                auto load_batch = [&](int zl, int yb, uint32_t (&buf)[C::NBR][V]) {
                    const uint32_t z = bz * B + zl;
#pragma unroll
                    for (int i = 0; i < C::NBR; ++i) {
                        const uint32_t y = min(by * B + yb + i, ny - 1);  // clamped row
                        load_codes<V, NTC>(a.codes + ((uint64_t)z * ny + y) * nx + xl, buf[i]);
                    }
                    // keep the loads here: the scheduler would otherwise sink
                    // them to their first use and serialise memory and compute
                    __builtin_amdgcn_sched_barrier(0);
                };
                auto decode_batch = [&](int zl, int yb, uint32_t (&buf)[C::NBR][V]) {
                    dec_batch<DIM, B, V, C::NBR, false>(a, st, buf, yb, bz * B + zl, by * B + yb, x0, xin, gmask, lane,
                                                 corrupt);
                };
                uint32_t bufA[C::NBR][V], bufB[C::NBR][V];
                if constexpr (DIM == 3 && YB == 2) {
                    const int nzl = (int)min((uint32_t)B, nz - bz * B);
                    load_batch(0, 0, bufA);
                    for (int zl = 0; zl < nzl; ++zl) {
                        load_batch(zl, C::NBR, bufB);
                        decode_batch(zl, 0, bufA);
                        if (zl + 1 < nzl) load_batch(zl + 1, 0, bufA);
                        decode_batch(zl, C::NBR, bufB);
                    }
                } else {
                    const int nbt = DIM == 3 ? (int)min((uint32_t)B, nz - bz * B)
                                             : (int)((min((uint32_t)B, ny - by * B) + C::NBR - 1) / C::NBR);
                    load_batch(0, 0, bufA);
                    for (int b = 0; b < nbt; b += 2) {
                        if (b + 1 < nbt) load_batch((b + 1) / YB, ((b + 1) % YB) * C::NBR, bufB);
                        decode_batch(b / YB, (b % YB) * C::NBR, bufA);
                        if (b + 1 < nbt) {
                            if (b + 2 < nbt) load_batch((b + 2) / YB, ((b + 2) % YB) * C::NBR, bufA);
                            decode_batch((b + 1) / YB, ((b + 1) % YB) * C::NBR, bufB);
                        }
                    }
                }
                if (leader && gvalid && st.rank != st.oe - st.os) corrupt = true;
            }
        }
    } else {
        const uint32_t R = (uint32_t)a.R;
        for (int bi = 0; bi < C::BPT; ++bi) {
            const uint32_t bx = tx * C::BPT + bi;
            if (bx >= a.g.nbx) break;
            uint32_t os = 0, oe = 0;
            if (a.n_out) block_run(a, bx, os, oe);
            const uint32_t peff = block_peff<DIM>(a, bx);
            uint32_t rank = 0, carry = 0;
            for (int cb = 0; cb < C::NCH; cb += C::NBR) {
                if (bx * B + cb * C::CX >= nx) break;
                uint32_t c[C::NBR][V];
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const uint32_t x0 = bx * B + (cb + i) * C::CX + (uint32_t)lane * V;
                    load_codes<V, NTC>(a.codes + min(x0, nx - V), c[i]);
                }
#pragma unroll
                for (int i = 0; i < C::NBR; ++i) {
                    const uint32_t xc = bx * B + (cb + i) * C::CX;
                    if (xc >= nx) continue;  // uniform
                    const uint32_t x0 = xc + (uint32_t)lane * V;
                    const bool xin = x0 < nx;
                    uint32_t cc[V], d[V];
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        cc[j] = xin ? c[i][j] : R;
                        d[j] = cc[j] - R;
                    }
                    fetch_outliers<V>(a, cc, d, rank, os, oe, ~0ull, x0, corrupt);
                    uint32_t s[V];
                    s[0] = d[0];
#pragma unroll
                    for (int j = 1; j < V; ++j) s[j] = s[j - 1] + d[j];
                    const uint32_t incl = seg_scan_incl<64>(s[V - 1], lane);
                    const uint32_t excl = incl - s[V - 1] + carry;
                    carry += readlane(incl, 63);
                    float o[V];
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        const int32_t q = (int32_t)(s[j] + excl + peff);
                        o[j] = (float)((double)q * a.twoeb);
                    }
                    if (xin) store_f<V>(a.x_hat + x0, o);
                }
            }
            if (lane == 0 && rank != oe - os) corrupt = true;
        }
    }
    if (ballot(corrupt) && lane == 0) status_corrupt_tagged(a.res_word, a.tag);
}

template <int DIM, int B, int V, bool NTC>
__global__ __launch_bounds__(kThreads) void k_decode(DecArgs a) {
    const int wave = (int)uniform(threadIdx.x >> 6);  // scalar: tile math stays in SGPRs
    const int lane = threadIdx.x & 63;
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x) * kWaves + wave;
    if (t >= a.g.n_tiles) return;  // tile 0 (which initialises the result) always exists
    decode_tile<DIM, B, V, NTC>(a, t, lane);
}

// Persistent decode of a batch of fields of one configuration, draining the
// flattened (field, run of tiles) queue with a workgroup ticket as the batch
// encode does.
template <int DIM, int B, int V>
__global__ __launch_bounds__(kThreads) void k_decode_batch(const DecArgs* __restrict__ dec,
                                                           const uint4* __restrict__ units, uint32_t n_units,
                                                           unsigned int* ticket) {
    __shared__ uint32_t s_unit;
    const int wave = (int)uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (;;) {
        if (threadIdx.x == 0) s_unit = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t u = uniform(s_unit);
        __syncthreads();
        if (u >= n_units) break;
        const uint4 un = units[u];  // field, first tile, tiles
        const DecArgs& a = dec[uniform(un.x)];
        const uint32_t t0 = uniform(un.y), t1 = t0 + uniform(un.z);
        for (uint32_t t = t0 + (uint32_t)wave; t < t1; t += kWaves) decode_tile<DIM, B, V, false, true>(a, t, lane);
    }
}

#ifndef DQ_DIM
#error "dq_decode.hip is compiled once per DQ_DIM (1, 2, 3)"
#endif

// instantiated only for the configurations of this object's dimensionality
template <int D, int BB, int VV>
static bool try_launch_decode(int block, int v, const DecArgs& a, dim3 grid, hipStream_t stream, bool nt_codes) {
    if constexpr (D == DQ_DIM) {
        if (block == BB && v == VV) {
            if (nt_codes)
                hipLaunchKernelGGL((k_decode<D, BB, VV, true>), grid, dim3(kThreads), 0, stream, a);
            else
                hipLaunchKernelGGL((k_decode<D, BB, VV, false>), grid, dim3(kThreads), 0, stream, a);
            return true;
        }
    }
    return false;
}

#define DQ_DEC_CASE(D, BB, VV) \
    if (try_launch_decode<D, BB, VV>(block, v, a, grid, stream, nt_codes)) return true;

bool DQ_CAT(launch_decode_dim, DQ_DIM)(int block, int v, const DecArgs& a, dim3 grid, hipStream_t stream,
                                       bool nt_codes) {
    DQ_CONFIGS(DQ_DEC_CASE)
    return false;
}

template <int D, int BB, int VV>
static bool try_launch_decode_batch(int block, int v, const BatchQueue& q, int grid, hipStream_t stream) {
    if constexpr (D == DQ_DIM) {
        if (block == BB && v == VV) {
            int per_cu = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(
                    &k_decode_batch<D, BB, VV>), kThreads, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            const int resident = per_cu * cus;
            hipLaunchKernelGGL((k_decode_batch<D, BB, VV>), dim3((uint32_t)(grid < resident ? grid : resident)),
                               dim3(kThreads), 0, stream, q.dec, q.units, q.n_units, q.ticket);
            return true;
        }
    }
    return false;
}

#define DQ_DECB_CASE(D, BB, VV) \
    if (try_launch_decode_batch<D, BB, VV>(block, v, q, grid, stream)) return true;

bool DQ_CAT(launch_decode_batch_dim, DQ_DIM)(int block, int v, const BatchQueue& q, int grid, hipStream_t stream) {
    DQ_CONFIGS(DQ_DECB_CASE)
    return false;
}

}  // namespace dq
