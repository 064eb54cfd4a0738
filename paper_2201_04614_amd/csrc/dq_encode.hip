// dq_encode.hip - fused dual-quantisation encode kernel (gfx950).
//
// One pass over x per tile (see dq_device.hpp for the tiling):
//   load V fp32 per lane (coalesced) -> q = round(x / 2eb)          (Section III-A)
//   -> zero-padded Lorenzo difference along x (DPP wave_shr:1), then y and z
//      against the previous row / plane kept in registers
//   -> code = delta + R or 0                                          (Section III-A)
//   -> uint16 stores; outliers found with ballots, ranked inside their block
//      and staged in LDS, flushed to a global staging list
//   -> at the end of each block: padding statistics (Section IV), the origin
//      residual q_o - P_eff (the only residual that depends on the padding,
//      because a face-constant halo cancels in every other Lorenzo
//      difference), per-block outlier bookkeeping.
// A later scan over tiles and a scatter put the staged outliers in
// block-major order.
#include "dq_device.hpp"
#include "dq_kernels.hpp"

namespace dq {

template <int DIM, int B, int V>
__global__ __launch_bounds__(kThreads) void k_encode(EncArgs a) {
    using C = Cfg<DIM, B, V>;
    __shared__ uint4 sbuf_all[kWaves][kStageCap];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint4* sbuf = sbuf_all[wave];
    const uint32_t t = blockIdx.x * kWaves + wave;
    if (t >= a.g.n_tiles) return;
    if (__builtin_nontemporal_load(a.status) != ST_OK) {
        if (lane == 0) a.tile_count[t] = 0;
        return;
    }
    const double r = a.sc->r, twoeb = a.sc->twoeb, eb = a.sc->eb;
    const uint32_t R = (uint32_t)a.R;
    const int pad = a.pad_mode;
    uint32_t gpad = 0;
    if (pad == PAD_GLOBAL) {
        gpad = (uint32_t)round_mean((long long)a.sc->sumq, (long long)a.g.N);
        if (t == 0 && lane == 0) a.pads[0] = (int32_t)gpad;
    }
    const uint32_t tx = t % a.g.ntx;
    const uint32_t rr = t / a.g.ntx;
    const uint32_t by = rr % a.g.nby;
    const uint32_t bz = rr / a.g.nby;
    const uint32_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;

    uint32_t scount = 0;      // LDS staged entries (wave-uniform)
    uint32_t tile_total = 0;  // outliers in this tile so far (wave-uniform)
    bool bad = false;         // |q| out of range or x not finite

    if constexpr (!C::WIDE) {
        const int gl = lane & (C::GPB - 1);
        const bool leader = gl == 0;
        const uint64_t gmask = (C::GPB == 64) ? ~0ull
                                              : (((1ull << C::GPB) - 1) << (lane & ~(C::GPB - 1)));
        for (int ch = 0; ch < C::XCH; ++ch) {
            const uint32_t bx0 = tx * C::BPT + ch * C::BPC;
            if (bx0 >= a.g.nbx) break;
            const uint32_t bx = bx0 + (uint32_t)(lane / C::GPB);
            const bool gvalid = bx < a.g.nbx;
            const uint32_t x0 = bx0 * B + (uint32_t)lane * V;
            const bool xin = x0 < nx;
            const uint32_t blk = (bz * a.g.nby + by) * a.g.nbx + bx;

            uint32_t rank = 0;  // non-origin outliers found so far in this block
            long long s_all = 0, s_fx = 0, s_fy = 0, s_fz = 0;
            uint32_t qo = 0;
            uint32_t dcode[V];
            uint32_t pY[V];
            uint32_t pZ[C::BY][V];
#pragma unroll
            for (int j = 0; j < V; ++j) { dcode[j] = 0; pY[j] = 0; }

            for (int zl = 0; zl < C::BZ; ++zl) {
                const uint32_t z = bz * B + zl;
                if (z >= nz) break;
#pragma unroll
                for (int yl = 0; yl < C::BY; ++yl) {
                    const uint32_t y = by * B + yl;
                    if (y >= ny) continue;  // uniform: rows past the field edge
                    const uint64_t row = ((uint64_t)z * ny + y) * nx;
                    float xv[V];
                    if (xin) {
                        load_f<V>(a.x + row + x0, xv);
                    } else {
#pragma unroll
                        for (int j = 0; j < V; ++j) xv[j] = 0.0f;
                    }
                    uint32_t q[V];
                    prequant<V>(xv, r, twoeb, eb, q, bad);
                    // Lorenzo residual with zero padding, separably: x, then y, then z
                    const uint32_t left = wave_shr1(q[V - 1]);
                    uint32_t d[V];
                    d[0] = q[0] - (leader ? 0u : left);
#pragma unroll
                    for (int j = 1; j < V; ++j) d[j] = q[j] - q[j - 1];
                    if constexpr (DIM >= 2) {
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            const uint32_t cur = d[j];
                            d[j] = (yl == 0) ? cur : cur - pY[j];
                            pY[j] = cur;
                        }
                    }
                    if constexpr (DIM == 3) {
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            const uint32_t cur = d[j];
                            d[j] = (zl == 0) ? cur : cur - pZ[yl][j];
                            pZ[yl][j] = cur;
                        }
                    }
                    // post-quantisation
                    const bool orow = (zl == 0) && (yl == 0);
                    uint32_t code[V];
                    bool out[V];
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        const uint32_t u = d[j] + (R - 1u);
                        const bool inl = u < 2u * R - 1u;
                        code[j] = inl ? u + 1u : 0u;
                        out[j] = xin && !inl;
                    }
                    if (orow && leader) out[0] = false;  // classified at the end of the block
                    // padding statistics (Section IV-A: mean of the data)
                    if (pad == PAD_BLOCK) {
                        if (xin) {
#pragma unroll
                            for (int j = 0; j < V; ++j) s_all += (int32_t)q[j];
                        }
                    } else if (pad == PAD_EDGE) {
                        if (xin) {
                            if (leader) s_fx += (int32_t)q[0];
                            if (DIM >= 2 && yl == 0) {
#pragma unroll
                                for (int j = 0; j < V; ++j) s_fy += (int32_t)q[j];
                            }
                            if (DIM == 3 && zl == 0) {
#pragma unroll
                                for (int j = 0; j < V; ++j) s_fz += (int32_t)q[j];
                            }
                        }
                    }
                    if (orow && leader) {
                        qo = q[0];
#pragma unroll
                        for (int j = 0; j < V; ++j) dcode[j] = code[j];
                    } else if (xin) {
                        store_codes<V>(a.codes + row + x0, code);
                    }
                    // outliers: rare path
                    uint64_t m[V];
                    uint64_t any = 0;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        m[j] = ballot(out[j]);
                        any |= m[j];
                    }
                    if (any) {
                        uint32_t tot = 0, below = 0, gtot = 0;
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            tot += popc(m[j]);
                            below += mbcnt(m[j] & gmask);
                            gtot += popc(m[j] & gmask);
                        }
                        if (scount + tot > (uint32_t)kStageCap) {
                            flush_stage(sbuf, scount, a.stage, a.stage_cap, &a.sc->stage_count, lane);
                            scount = 0;
                        }
                        uint32_t slot = scount, own = 0;
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            if (out[j]) {
                                sbuf[slot + mbcnt(m[j])] =
                                    make_uint4((uint32_t)(row + x0 + j), d[j], blk, rank + below + own);
                                ++own;
                            }
                            slot += popc(m[j]);
                        }
                        scount += tot;
                        rank += gtot;
                    }
                }
            }

            // ---- end of the blocks of this step: padding and origins
            uint32_t peff = 0;
            if (pad == PAD_GLOBAL) {
                peff = gpad;
            } else if (pad != PAD_ZERO) {
                const long long ex = (long long)min((uint32_t)B, nx - min(nx, bx * B));
                const long long ey = DIM >= 2 ? (long long)min((uint32_t)B, ny - by * B) : 1;
                const long long ez = DIM == 3 ? (long long)min((uint32_t)B, nz - bz * B) : 1;
                if (pad == PAD_BLOCK) {
                    const long long S = group_sum64<C::GPB>(s_all);
                    const int32_t P = round_mean(S, gvalid ? ex * ey * ez : 1);
                    peff = (uint32_t)P;
                    if (leader && gvalid) a.pads[blk] = P;
                } else {
                    const long long Sx = group_sum64<C::GPB>(s_fx);
                    int32_t e[3] = {0, 0, 0};
                    if constexpr (DIM == 1) {
                        e[0] = (int32_t)qo;  // the x face of a 1-D block is its first cell
                    } else if constexpr (DIM == 2) {
                        const long long Sy = group_sum64<C::GPB>(s_fy);
                        e[0] = round_mean(Sy, gvalid ? ex : 1);  // axis 0 (y): first row
                        e[1] = round_mean(Sx, ey);               // axis 1 (x): first column
                    } else {
                        const long long Sy = group_sum64<C::GPB>(s_fy);
                        const long long Sz = group_sum64<C::GPB>(s_fz);
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
                od = qo - peff;
                const uint32_t u = od + (R - 1u);
                const bool inl = u < 2u * R - 1u;
                dcode[0] = inl ? u + 1u : 0u;
                oout = !inl;
                store_codes<V>(a.codes + orow_base + x0, dcode);
            }
            const uint64_t mo = ballot(oout);
            if (mo) {
                const uint32_t n = popc(mo);
                if (scount + n > (uint32_t)kStageCap) {
                    flush_stage(sbuf, scount, a.stage, a.stage_cap, &a.sc->stage_count, lane);
                    scount = 0;
                }
                if (oout)
                    sbuf[scount + mbcnt(mo)] = make_uint4((uint32_t)(orow_base + x0), od, blk, kOriginFlag);
                scount += n;
            }
            // per-block outlier counts -> exclusive prefix inside the tile
            const uint32_t cnt = (leader && gvalid) ? rank + (oout ? 1u : 0u) : 0u;
            uint32_t excl = 0, step_total = 0;
            if (ballot(cnt != 0)) {
                const uint32_t incl = wave_scan_incl(cnt, lane);
                excl = incl - cnt;
                step_total = readlane(incl, 63);
            }
            if (leader && gvalid) a.block_info[blk] = (tile_total + excl) | (oout ? kOriginFlag : 0u);
            tile_total += step_total;
        }
    } else {
        // 1-D blocks wider than one wave step: blocks one after another
        const uint32_t nblk = a.g.nbx;
        for (int bi = 0; bi < C::BPT; ++bi) {
            const uint32_t bx = tx * C::BPT + bi;
            if (bx >= nblk) break;
            uint32_t rank = 0, carry = 0, qo = 0;
            long long s_all = 0;
            uint32_t dcode[V];
#pragma unroll
            for (int j = 0; j < V; ++j) dcode[j] = 0;
            for (int ch = 0; ch < C::NCH; ++ch) {
                const uint32_t xc = bx * B + ch * C::CX;
                if (xc >= nx) break;
                const uint32_t x0 = xc + (uint32_t)lane * V;
                const bool xin = x0 < nx;
                float xv[V];
                if (xin) {
                    load_f<V>(a.x + x0, xv);
                } else {
#pragma unroll
                    for (int j = 0; j < V; ++j) xv[j] = 0.0f;
                }
                uint32_t q[V];
                prequant<V>(xv, r, twoeb, eb, q, bad);
                uint32_t left = wave_shr1(q[V - 1]);
                if (lane == 0) left = carry;  // 0 at the block start
                carry = readlane(q[V - 1], 63);
                uint32_t d[V];
                d[0] = q[0] - left;
#pragma unroll
                for (int j = 1; j < V; ++j) d[j] = q[j] - q[j - 1];
                const bool origin_lane = (ch == 0) && (lane == 0);
                uint32_t code[V];
                bool out[V];
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const uint32_t u = d[j] + (R - 1u);
                    const bool inl = u < 2u * R - 1u;
                    code[j] = inl ? u + 1u : 0u;
                    out[j] = xin && !inl;
                }
                if (origin_lane) out[0] = false;
                if (pad == PAD_BLOCK && xin) {
#pragma unroll
                    for (int j = 0; j < V; ++j) s_all += (int32_t)q[j];
                }
                if (origin_lane) {
                    qo = q[0];
#pragma unroll
                    for (int j = 0; j < V; ++j) dcode[j] = code[j];
                } else if (xin) {
                    store_codes<V>(a.codes + x0, code);
                }
                uint64_t m[V];
                uint64_t any = 0;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    m[j] = ballot(out[j]);
                    any |= m[j];
                }
                if (any) {
                    uint32_t tot = 0, below = 0;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        tot += popc(m[j]);
                        below += mbcnt(m[j]);
                    }
                    if (scount + tot > (uint32_t)kStageCap) {
                        flush_stage(sbuf, scount, a.stage, a.stage_cap, &a.sc->stage_count, lane);
                        scount = 0;
                    }
                    uint32_t slot = scount, own = 0;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        if (out[j]) {
                            sbuf[slot + mbcnt(m[j])] = make_uint4(x0 + j, d[j], bx, rank + below + own);
                            ++own;
                        }
                        slot += popc(m[j]);
                    }
                    scount += tot;
                    rank += tot;
                }
            }
            uint32_t peff = 0;
            if (pad == PAD_GLOBAL) {
                peff = gpad;
            } else if (pad == PAD_BLOCK) {
                const long long S = group_sum64<64>(s_all);
                const long long ex = (long long)min((uint32_t)B, nx - bx * B);
                const int32_t P = round_mean(S, ex);
                peff = (uint32_t)P;
                if (lane == 0) a.pads[bx] = P;
            } else if (pad == PAD_EDGE) {
                peff = readlane(qo, 0);
                if (lane == 0) a.pads[bx] = (int32_t)peff;
            }
            bool oout = false;
            uint32_t od = 0;
            if (lane == 0) {
                od = qo - peff;
                const uint32_t u = od + (R - 1u);
                const bool inl = u < 2u * R - 1u;
                dcode[0] = inl ? u + 1u : 0u;
                oout = !inl;
                store_codes<V>(a.codes + (uint64_t)bx * B, dcode);
            }
            if (ballot(oout)) {
                if (scount + 1 > (uint32_t)kStageCap) {
                    flush_stage(sbuf, scount, a.stage, a.stage_cap, &a.sc->stage_count, lane);
                    scount = 0;
                }
                if (lane == 0) sbuf[scount] = make_uint4(bx * B, od, bx, kOriginFlag);
                scount += 1;
            }
            const uint32_t cnt = readlane(rank + (oout ? 1u : 0u), 0);
            if (lane == 0) a.block_info[bx] = tile_total | (oout ? kOriginFlag : 0u);
            tile_total += cnt;
        }
    }

    if (scount) flush_stage(sbuf, scount, a.stage, a.stage_cap, &a.sc->stage_count, lane);
    if (lane == 0) a.tile_count[t] = tile_total;
    if (ballot(bad) && lane == 0) __hip_atomic_store(a.status, ST_ERANGE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

#define DQ_ENC_CASE(D, BB, VV)                                              \
    if (dim == D && block == BB && v == VV) {                               \
        hipLaunchKernelGGL((k_encode<D, BB, VV>), grid, dim3(kThreads), 0, stream, a); \
        return true;                                                        \
    }

bool launch_encode(int dim, int block, int v, const EncArgs& a, dim3 grid, hipStream_t stream) {
    DQ_CONFIGS(DQ_ENC_CASE)
    return false;
}

#define DQ_BPT_CASE(D, BB, VV) \
    if (dim == D && block == BB && v == VV) return Cfg<D, BB, VV>::BPT;

int tile_blocks(int dim, int block, int v) {
    DQ_CONFIGS(DQ_BPT_CASE)
    return 0;
}

}  // namespace dq
