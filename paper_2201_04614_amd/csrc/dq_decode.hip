// dq_decode.hip - fused dual-quantisation decode kernel (gfx950).
//
// Decompression reverses the prediction (Section III-A). The residual of the
// zero-padded Lorenzo predictor is the mixed backward difference along every
// axis, so its inverse inside a block is the n-D inclusive prefix sum; the
// padding enters only through the block origin, so
//     q(u) = P_eff + sum_{w <= u, same block} delta(w).
// Per tile and row: load V uint16 codes per lane, delta = code - R (or the
// outlier value, looked up by its rank inside the block), in-lane prefix over
// the V cells, segmented DPP scan over the GPB lanes of each block row,
// running sums over rows (y) and planes (z) in registers, add P_eff, and
// dequantise x_hat = (float)((double)q * 2eb) with one fp64 product.
#include "dq_device.hpp"
#include "dq_kernels.hpp"

namespace dq {

template <int DIM>
__device__ __forceinline__ uint32_t block_peff(const DecArgs& a, uint32_t blk) {
    const int pad = a.pad_mode;
    if (pad == PAD_ZERO) return 0u;
    if (pad == PAD_GLOBAL) return (uint32_t)a.pads[0];
    if (pad == PAD_BLOCK) return (uint32_t)a.pads[blk];
    int32_t e[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) e[k] = a.pads[(uint64_t)blk * DIM + k];
    return edge_effective<DIM>(e);
}

__device__ __forceinline__ void mark_corrupt(int32_t* status) {
    __hip_atomic_store(status, ST_ECORRUPT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DIM, int B, int V>
__global__ __launch_bounds__(kThreads) void k_decode(DecArgs a) {
    using C = Cfg<DIM, B, V>;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * kWaves + wave;
    if (t >= a.g.n_tiles) return;
    const uint32_t R = (uint32_t)a.R;
    const double twoeb = a.twoeb;
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
        for (int ch = 0; ch < C::XCH; ++ch) {
            const uint32_t bx0 = tx * C::BPT + ch * C::BPC;
            if (bx0 >= a.g.nbx) break;
            const uint32_t bx = bx0 + (uint32_t)(lane / C::GPB);
            const bool gvalid = bx < a.g.nbx;
            const uint32_t x0 = bx0 * B + (uint32_t)lane * V;
            const bool xin = x0 < nx;
            const uint32_t blk = (bz * a.g.nby + by) * a.g.nbx + bx;
            uint32_t os = 0, oe = 0;
            if (a.n_out && gvalid) {
                os = a.block_start[blk];
                oe = a.block_start[blk + 1];
            }
            const uint32_t peff = gvalid ? block_peff<DIM>(a, blk) : 0u;
            uint32_t rank = 0;
            uint32_t pY[V];
            uint32_t pZ[C::BY][V];
#pragma unroll
            for (int j = 0; j < V; ++j) pY[j] = 0;
#pragma unroll
            for (int k = 0; k < C::BY; ++k)
#pragma unroll
                for (int j = 0; j < V; ++j) pZ[k][j] = 0;

            for (int zl = 0; zl < C::BZ; ++zl) {
                const uint32_t z = bz * B + zl;
                if (z >= nz) break;
#pragma unroll
                for (int yl = 0; yl < C::BY; ++yl) {
                    const uint32_t y = by * B + yl;
                    if (y >= ny) continue;  // uniform: rows past the field edge
                    const uint64_t row = ((uint64_t)z * ny + y) * nx;
                    uint32_t c[V];
                    if (xin) {
                        load_codes<V>(a.codes + row + x0, c);
                    } else {
#pragma unroll
                        for (int j = 0; j < V; ++j) c[j] = R;
                    }
                    uint32_t d[V];
                    uint64_t m[V];
                    uint64_t any = 0;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        d[j] = c[j] - R;
                        m[j] = ballot(c[j] == 0u);
                        any |= m[j];
                    }
                    if (any) {  // outliers: k-th zero code of a block is its k-th outlier
                        uint32_t below = 0, gtot = 0, own = 0;
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            below += mbcnt(m[j] & gmask);
                            gtot += popc(m[j] & gmask);
                        }
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            if (c[j] == 0u) {
                                const uint32_t k = os + rank + below + own;
                                ++own;
                                const uint32_t gi = (uint32_t)(row + x0 + j);
                                if (k < oe && a.out_idx[k] == gi) {
                                    d[j] = (uint32_t)a.out_val[k];
                                } else {
                                    corrupt = true;
                                    d[j] = 0;
                                }
                            }
                        }
                        rank += gtot;
                    }
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
                            p = (yl == 0) ? p : p + pY[j];
                            pY[j] = p;
                        }
                        if constexpr (DIM == 3) {
                            p = p + pZ[yl][j];
                            pZ[yl][j] = p;
                        }
                        const int32_t q = (int32_t)(p + peff);
                        o[j] = (float)((double)q * twoeb);
                    }
                    if (xin) store_f<V>(a.x_hat + row + x0, o);
                }
            }
            if (leader && gvalid && rank != oe - os) corrupt = true;
        }
    } else {
        for (int bi = 0; bi < C::BPT; ++bi) {
            const uint32_t bx = tx * C::BPT + bi;
            if (bx >= a.g.nbx) break;
            uint32_t os = 0, oe = 0;
            if (a.n_out) {
                os = a.block_start[bx];
                oe = a.block_start[bx + 1];
            }
            const uint32_t peff = block_peff<DIM>(a, bx);
            uint32_t rank = 0, carry = 0;
            for (int ch = 0; ch < C::NCH; ++ch) {
                const uint32_t xc = bx * B + ch * C::CX;
                if (xc >= nx) break;
                const uint32_t x0 = xc + (uint32_t)lane * V;
                const bool xin = x0 < nx;
                uint32_t c[V];
                if (xin) {
                    load_codes<V>(a.codes + x0, c);
                } else {
#pragma unroll
                    for (int j = 0; j < V; ++j) c[j] = R;
                }
                uint32_t d[V];
                uint64_t m[V];
                uint64_t any = 0;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    d[j] = c[j] - R;
                    m[j] = ballot(c[j] == 0u);
                    any |= m[j];
                }
                if (any) {
                    uint32_t below = 0, tot = 0, own = 0;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        below += mbcnt(m[j]);
                        tot += popc(m[j]);
                    }
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        if (c[j] == 0u) {
                            const uint32_t k = os + rank + below + own;
                            ++own;
                            if (k < oe && a.out_idx[k] == x0 + j) {
                                d[j] = (uint32_t)a.out_val[k];
                            } else {
                                corrupt = true;
                                d[j] = 0;
                            }
                        }
                    }
                    rank += tot;
                }
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
                    o[j] = (float)((double)q * twoeb);
                }
                if (xin) store_f<V>(a.x_hat + x0, o);
            }
            if (lane == 0 && rank != oe - os) corrupt = true;
        }
    }
    if (ballot(corrupt) && lane == 0) mark_corrupt(a.status);
}

#define DQ_DEC_CASE(D, BB, VV)                                              \
    if (dim == D && block == BB && v == VV) {                               \
        hipLaunchKernelGGL((k_decode<D, BB, VV>), grid, dim3(kThreads), 0, stream, a); \
        return true;                                                        \
    }

bool launch_decode(int dim, int block, int v, const DecArgs& a, dim3 grid, hipStream_t stream) {
    DQ_CONFIGS(DQ_DEC_CASE)
    return false;
}

}  // namespace dq
