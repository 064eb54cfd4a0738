// dq_select.hip - per-block padding / block-size selector (gfx950).
//
//  k_block_stats      one wave per block: q = round(x / 2eb) of every cell and
//                     of its in-block lower neighbours (the codec's own exact
//                     pre-quantisation), integer sums / extremes / faces /
//                     roughness, zero codes away from the origin
//  k_block_select     one thread per block: five candidate pads (Section IV-A
//                     statistics at block and global granularity, the edge
//                     values of Section IV-B folded into the origin's
//                     effective pad), their origin outlier flags (pad
//                     locality: only q_o - P_eff depends on the pad), the
//                     exhaustive label and 24 features
//  k_super_cost       8 * outliers + 4 per block, summed per 16^d super-block
//  k_mlp_tile         fused forward + backward of the 24-64-64-8 network for
//                     32 samples, weights and activations in LDS, partial
//                     gradients per tile (reduced in a fixed order)
//  k_mlp_infer_bf16   bf16 weights / activations, fp32 accumulation
// The network is small (6280 parameters, 64-wide layers): its products are
// latency-bound FMA loops over LDS, not tiles for the matrix cores.
#include <climits>
#include <cmath>

#include "dq_device.hpp"
#include "dq_select.h"

namespace dq {
namespace {

constexpr int kFeat = DQ_SEL_FEATURES, kHid = DQ_SEL_HIDDEN, kOut = DQ_SEL_OUTPUTS, kCand = DQ_SEL_CANDIDATES;
constexpr int kNPad = 5, kNBsz = 3;
constexpr int kParams = DQ_MLP_PARAMS;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kFeat, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kOut * kHid;
static_assert(oB3 + kOut == kParams, "parameter layout");
constexpr double kClamp = 8.0;

// 3-D view of a 1-, 2- or 3-D field: axis 0 (z) slowest, leading extents 1.
struct SelGeom {
    uint32_t n[3];   // extents (z, y, x)
    uint32_t nb[3];  // blocks per axis
    uint32_t B, d, lb;
    uint32_t nsb[3];  // 16^d super-blocks per axis
    uint64_t N, nblocks;
};

bool make_sel_geom(const dq_params* p, SelGeom& g) {
    if (!p || p->ndim < 1 || p->ndim > 3 || p->block < 1) return false;
    const int d = p->ndim;
    g.d = (uint32_t)d;
    g.B = (uint32_t)p->block;
    g.lb = 0;
    while ((1u << g.lb) < g.B) ++g.lb;
    g.N = 1;
    g.nblocks = 1;
    for (int a = 0; a < 3; ++a) {
        const int fa = a - (3 - d);  // field axis of view axis a
        g.n[a] = fa >= 0 ? (uint32_t)p->shape[fa] : 1u;
        if (fa >= 0 && (p->shape[fa] < 1 || p->shape[fa] > 0xffffffffll)) return false;
        g.nb[a] = fa >= 0 ? (g.n[a] + g.B - 1) / g.B : 1u;
        g.nsb[a] = fa >= 0 ? (g.n[a] + DQ_SEL_SUPER - 1) / DQ_SEL_SUPER : 1u;
        g.N *= g.n[a];
        g.nblocks *= g.nb[a];
    }
    return g.N <= 0xffffffffull;
}

struct BlockBox {
    uint32_t o[3];    // origin (z, y, x)
    uint32_t ext[3];  // extents, 1 on absent axes
    uint32_t cells;
};

__device__ __forceinline__ BlockBox block_box(const SelGeom& g, uint64_t b) {
    BlockBox bb;
    const uint32_t bx = (uint32_t)(b % g.nb[2]);
    const uint64_t r = b / g.nb[2];
    const uint32_t by = (uint32_t)(r % g.nb[1]);
    const uint32_t bz = (uint32_t)(r / g.nb[1]);
    const uint32_t bc[3] = {bz, by, bx};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bb.o[a] = bc[a] * g.B;
        bb.ext[a] = min(g.B, g.n[a] - bb.o[a]);
    }
    bb.cells = bb.ext[0] * bb.ext[1] * bb.ext[2];
    return bb;
}

// ------------------------------------------------------------------ statistics

__global__ __launch_bounds__(256) void k_block_stats(SelGeom g, const float* __restrict__ x,
                                                     const uint16_t* __restrict__ codes, double r, double twoeb,
                                                     double eb, dq_block_stat* __restrict__ stats,
                                                     int32_t* status) {
    const int lane = threadIdx.x & 63;
    const uint64_t b = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    if (b >= g.nblocks) return;  // wave-uniform
    const BlockBox bb = block_box(g, b);
    const uint64_t sy = g.n[2], sz = (uint64_t)g.n[2] * g.n[1];
    const uint64_t o = bb.o[0] * sz + bb.o[1] * sy + bb.o[2];
    uint64_t bad = 0;
    float xo[1] = {x[o]};
    uint32_t qo1[1];
    prequant<1>(xo, r, twoeb, eb, qo1, bad);
    const int32_t qo = (int32_t)qo1[0];
    long long s = 0, mad = 0, fs[3] = {0, 0, 0}, rg[3] = {0, 0, 0};
    int32_t mn = INT_MAX, mx = INT_MIN;
    uint32_t nz = 0;
    const uint32_t exy = bb.ext[2] * bb.ext[1];
    const uint32_t iters = (bb.cells + 63u) / 64u;
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t k = it * 64u + (uint32_t)lane;
        const bool valid = k < bb.cells;
        const uint32_t kk = valid ? k : 0u;  // every lane takes part in the rounding's ballots
        const uint32_t u[3] = {kk / exy, (kk / bb.ext[2]) % bb.ext[1], kk % bb.ext[2]};
        const uint64_t gi = o + u[0] * sz + u[1] * sy + u[2];
        float xv[4];
        xv[0] = x[gi];
        xv[1] = x[u[0] ? gi - sz : gi];  // lower neighbour along z, y, x (in the block)
        xv[2] = x[u[1] ? gi - sy : gi];
        xv[3] = x[u[2] ? gi - 1 : gi];
        uint32_t q[4];
        prequant<4>(xv, r, twoeb, eb, q, bad);
        if (valid) {
            const int32_t v = (int32_t)q[0];
            s += v;
            mn = min(mn, v);
            mx = max(mx, v);
            mad += llabs((long long)v - qo);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                fs[a] += u[a] == 0 ? (long long)v : 0ll;
                rg[a] += u[a] != 0 ? llabs((long long)v - (int32_t)q[1 + a]) : 0ll;
            }
            if (codes && k > 0 && codes[gi] == 0) ++nz;
        }
    }
    s = group_sum64<64>(s);
    mad = group_sum64<64>(mad);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        fs[a] = group_sum64<64>(fs[a]);
        rg[a] = group_sum64<64>(rg[a]);
    }
    mn = group_min32<64>(mn);
    mx = group_max32<64>(mx);
    nz = (uint32_t)group_sum64<64>((long long)nz);
    if (lane == 0) {
        dq_block_stat st;
        st.qo = qo;
        st.mn = mn;
        st.mx = mx;
        st.nonorig = nz;
        st.sum = s;
        st.mad = mad;
        for (int a = 0; a < 3; ++a) {  // field axis a = view axis a + 3 - d
            const int va = a + 3 - (int)g.d;
            st.fsum[a] = a < (int)g.d ? fs[va] : 0;
            st.rough[a] = a < (int)g.d ? rg[va] : 0;
        }
        stats[b] = st;
        if (bad && status) __hip_atomic_store(status, ST_ERANGE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ candidates and features

__global__ void k_zero64(long long* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ __launch_bounds__(256) void k_sum_blocks(const dq_block_stat* __restrict__ st, uint64_t nb,
                                                    long long* gsum) {
    __shared__ long long red[4];
    long long s = 0;
    for (uint64_t b = (uint64_t)blockIdx.x * 256u + threadIdx.x; b < nb; b += (uint64_t)gridDim.x * 256u)
        s += st[b].sum;
    s = group_sum64<64>(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(gsum),
                  (unsigned long long)(red[0] + red[1] + red[2] + red[3]));
}

__device__ __forceinline__ float clampf(double v) {
    return (float)__builtin_fmin(__builtin_fmax(v, -kClamp), kClamp);
}

__device__ __forceinline__ int32_t edge_eff_d(const int32_t* e, int d) {
    if (d == 1) return (int32_t)edge_effective<1>(e);
    if (d == 2) return (int32_t)edge_effective<2>(e);
    return (int32_t)edge_effective<3>(e);
}

__global__ __launch_bounds__(256) void k_block_select(SelGeom g, const dq_block_stat* __restrict__ stats,
                                                      const long long* __restrict__ gsum, int32_t R,
                                                      int32_t* __restrict__ cand, uint8_t* __restrict__ flags,
                                                      int32_t* __restrict__ label, float* __restrict__ feat) {
    const uint64_t b = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (b >= g.nblocks) return;
    const int d = (int)g.d;
    const dq_block_stat st = stats[b];
    const BlockBox bb = block_box(g, b);
    const long long cells = bb.cells;
    const int32_t gmean = round_mean(*gsum, (long long)g.N);
    const int32_t bmean = round_mean(st.sum, cells);
    int32_t e[3] = {0, 0, 0};
    long long npairs[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
        const long long ext = bb.ext[a + 3 - d];
        e[a] = round_mean(st.fsum[a], cells / ext);
        npairs[a] = cells - cells / ext;
    }
    const int32_t c[kCand] = {0, gmean, bmean, edge_eff_d(e, d), round_mean((long long)st.mn + st.mx, 2)};
    uint32_t fl = 0;
    int32_t lab = -1;
    int32_t dl[kCand];
#pragma unroll
    for (int k = 0; k < kCand; ++k) {
        dl[k] = (int32_t)((uint32_t)st.qo - (uint32_t)c[k]);  // the origin residual, modulo 2^32
        const bool out = !(dl[k] > -R && dl[k] < R);
        fl |= out ? (1u << k) : 0u;
        if (!out && lab < 0) lab = k;
        if (cand) cand[b * kCand + k] = c[k];
    }
    if (flags) flags[b] = (uint8_t)fl;
    if (label) label[b] = lab < 0 ? 0 : lab;
    if (feat) {
        const double Rd = (double)R;
        float f[kFeat];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) f[k] = 0.0f;
#pragma unroll
        for (int k = 0; k < kCand; ++k) {
            f[k] = clampf((double)dl[k] / Rd);
            f[kCand + k] = clampf(__builtin_fabs((double)dl[k]) / Rd);
        }
        f[10] = clampf((double)((long long)st.mx - st.mn) / Rd);
        f[11] = clampf((double)((long long)bmean - gmean) / Rd);
        for (int a = 0; a < d; ++a) {
            f[12 + a] = clampf((double)((long long)e[a] - bmean) / Rd);
            if (npairs[a] > 0) f[18 + a] = clampf((double)st.rough[a] / ((double)npairs[a] * Rd));
        }
        f[15] = clampf((double)((long long)st.qo - st.mn) / Rd);
        f[16] = clampf((double)((long long)st.mx - st.qo) / Rd);
        f[17] = clampf((double)st.mad / ((double)cells * Rd));
        f[21] = clampf((double)gmean / (64.0 * Rd));
        f[22] = (float)((double)d / 3.0);
        f[23] = (float)((double)g.lb / 4.0);
        float* out = feat + b * kFeat;
#pragma unroll
        for (int k = 0; k < kFeat; ++k) out[k] = f[k];
    }
}

__global__ __launch_bounds__(256) void k_super_cost(SelGeom g, const dq_block_stat* __restrict__ stats,
                                                    const uint8_t* __restrict__ flags,
                                                    const int32_t* __restrict__ choice,
                                                    unsigned long long* __restrict__ cost) {
    const uint64_t b = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (b >= g.nblocks) return;
    const BlockBox bb = block_box(g, b);
    const uint64_t s = ((uint64_t)(bb.o[0] / DQ_SEL_SUPER) * g.nsb[1] + bb.o[1] / DQ_SEL_SUPER) * g.nsb[2] +
                       bb.o[2] / DQ_SEL_SUPER;
    const int32_t c = choice[b];
    const uint32_t o = (c >= 0 && c < kCand) ? ((flags[b] >> c) & 1u) : (flags[b] & 1u);
    atomicAdd(cost + s, 8ull * ((unsigned long long)stats[b].nonorig + o) + 4ull);
}

__global__ __launch_bounds__(256) void k_gather_pads(const int32_t* __restrict__ cand,
                                                     const int32_t* __restrict__ choice, uint64_t nb,
                                                     int32_t* __restrict__ pads) {
    const uint64_t b = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (b >= nb) return;
    const int32_t c = choice[b];
    pads[b] = cand[b * kCand + ((c >= 0 && c < kCand) ? c : 0)];
}

// ------------------------------------------------------------------ MLP training

constexpr int kTile = 32;            // samples per workgroup
constexpr int sF = kFeat + 1;        // padded LDS row strides
constexpr int sH = kHid + 1;

// Forward and backward of kTile samples; writes the tile's gradient sum
// (scaled by 1 / n) and its loss sum (scaled likewise).
__global__ __launch_bounds__(256) void k_mlp_tile(const float* __restrict__ theta, const float* __restrict__ X,
                                                  const int32_t* __restrict__ ypad,
                                                  const int32_t* __restrict__ ybsz, uint64_t n,
                                                  float* __restrict__ partial, float* __restrict__ lossp) {
    __shared__ float W1[kHid * sF], W2[kHid * sH], W3[kOut * sH], b1[kHid], b2[kHid], b3[kOut];
    __shared__ float sX[kTile * sF], H1[kTile * sH], H2[kTile * sH], D2[kTile * sH], D1[kTile * sH];
    __shared__ float DZ[kTile * kOut];
    __shared__ float sl[kTile];
    const int t = threadIdx.x;
    const uint64_t s0 = (uint64_t)blockIdx.x * kTile;
    const float inv_n = 1.0f / (float)n;
    for (int i = t; i < kHid * kFeat; i += 256) W1[(i / kFeat) * sF + i % kFeat] = theta[oW1 + i];
    for (int i = t; i < kHid * kHid; i += 256) W2[(i / kHid) * sH + i % kHid] = theta[oW2 + i];
    for (int i = t; i < kOut * kHid; i += 256) W3[(i / kHid) * sH + i % kHid] = theta[oW3 + i];
    if (t < kHid) {
        b1[t] = theta[oB1 + t];
        b2[t] = theta[oB2 + t];
    }
    if (t < kOut) b3[t] = theta[oB3 + t];
    for (int i = t; i < kTile * kFeat; i += 256) {
        const uint64_t s = s0 + (uint64_t)(i / kFeat);
        sX[(i / kFeat) * sF + i % kFeat] = s < n ? X[s * kFeat + i % kFeat] : 0.0f;
    }
    __syncthreads();
    const int j = t & 63, sr = t >> 6;  // output column, first sample row (rows sr + 4 i)
    // layer 1 and 2
    for (int i = 0; i < kTile / 4; ++i) {
        const int s = sr + 4 * i;
        float acc = b1[j];
        for (int k = 0; k < kFeat; ++k) acc += sX[s * sF + k] * W1[j * sF + k];
        H1[s * sH + j] = acc > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    for (int i = 0; i < kTile / 4; ++i) {
        const int s = sr + 4 * i;
        float acc = b2[j];
        for (int k = 0; k < kHid; ++k) acc += H1[s * sH + k] * W2[j * sH + k];
        H2[s * sH + j] = acc > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    {  // logits: one (sample, output) per thread
        const int s = t >> 3, o = t & 7;
        float acc = b3[o];
        for (int k = 0; k < kHid; ++k) acc += H2[s * sH + k] * W3[o * sH + k];
        DZ[s * kOut + o] = acc;
    }
    __syncthreads();
    if (t < kTile) {  // softmax cross-entropy of both heads
        const int s = t;
        const bool valid = s0 + (uint64_t)s < n;
        float* z = DZ + s * kOut;
        float l = 0.0f;
        if (valid) {
            const int yp = ypad[s0 + s], yb = ybsz[s0 + s];
            float m = z[0];
            for (int o = 1; o < kNPad; ++o) m = fmaxf(m, z[o]);
            float den = 0.0f;
            for (int o = 0; o < kNPad; ++o) den += expf(z[o] - m);
            const float lse_p = m + logf(den);
            float mb = z[kNPad];
            for (int o = 1; o < kNBsz; ++o) mb = fmaxf(mb, z[kNPad + o]);
            float denb = 0.0f;
            for (int o = 0; o < kNBsz; ++o) denb += expf(z[kNPad + o] - mb);
            const float lse_b = mb + logf(denb);
            l = (lse_p - z[yp]) + (lse_b - z[kNPad + yb]);
            for (int o = 0; o < kNPad; ++o) z[o] = (expf(z[o] - lse_p) - (o == yp ? 1.0f : 0.0f)) * inv_n;
            for (int o = 0; o < kNBsz; ++o)
                z[kNPad + o] = (expf(z[kNPad + o] - lse_b) - (o == yb ? 1.0f : 0.0f)) * inv_n;
        } else {
            for (int o = 0; o < kOut; ++o) z[o] = 0.0f;
        }
        sl[s] = l * inv_n;
    }
    __syncthreads();
    // back through layer 3 and 2
    for (int i = 0; i < kTile / 4; ++i) {
        const int s = sr + 4 * i;
        float acc = 0.0f;
        for (int o = 0; o < kOut; ++o) acc += DZ[s * kOut + o] * W3[o * sH + j];
        D2[s * sH + j] = H2[s * sH + j] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    for (int i = 0; i < kTile / 4; ++i) {
        const int s = sr + 4 * i;
        float acc = 0.0f;
        for (int k = 0; k < kHid; ++k) acc += D2[s * sH + k] * W2[k * sH + j];
        D1[s * sH + j] = H1[s * sH + j] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // parameter gradients of the tile (sums over its samples, in order)
    float* gp = partial + (uint64_t)blockIdx.x * kParams;
    for (int i = t; i < kHid * kFeat; i += 256) {
        const int r = i / kFeat, c = i % kFeat;
        float acc = 0.0f;
        for (int s = 0; s < kTile; ++s) acc += D1[s * sH + r] * sX[s * sF + c];
        gp[oW1 + i] = acc;
    }
    for (int i = t; i < kHid * kHid; i += 256) {
        const int r = i / kHid, c = i % kHid;
        float acc = 0.0f;
        for (int s = 0; s < kTile; ++s) acc += D2[s * sH + r] * H1[s * sH + c];
        gp[oW2 + i] = acc;
    }
    for (int i = t; i < kOut * kHid; i += 256) {
        const int r = i / kHid, c = i % kHid;
        float acc = 0.0f;
        for (int s = 0; s < kTile; ++s) acc += DZ[s * kOut + r] * H2[s * sH + c];
        gp[oW3 + i] = acc;
    }
    if (t < kHid) {
        float a1 = 0.0f, a2 = 0.0f;
        for (int s = 0; s < kTile; ++s) {
            a1 += D1[s * sH + t];
            a2 += D2[s * sH + t];
        }
        gp[oB1 + t] = a1;
        gp[oB2 + t] = a2;
    }
    if (t < kOut) {
        float a3 = 0.0f;
        for (int s = 0; s < kTile; ++s) a3 += DZ[s * kOut + t];
        gp[oB3 + t] = a3;
    }
    if (t == 0) {
        float l = 0.0f;
        for (int s = 0; s < kTile; ++s) l += sl[s];
        lossp[blockIdx.x] = l;
    }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, const float* __restrict__ lossp,
                                                    uint32_t tiles, float* __restrict__ grad, float* loss) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < (uint32_t)kParams) {
        float acc = 0.0f;
        for (uint32_t k = 0; k < tiles; ++k) acc += partial[(uint64_t)k * kParams + i];
        grad[i] = acc;
    }
    if (i == 0 && loss) {
        float l = 0.0f;
        for (uint32_t k = 0; k < tiles; ++k) l += lossp[k];
        *loss = l;
    }
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ theta, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ g, float lr,
                                                  float c1, float c2) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (uint32_t)kParams) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// ------------------------------------------------------------------ bf16 inference

__device__ __forceinline__ uint16_t to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // nearest, ties to even (finite values)
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float round_bf16(float f) { return from_bf16(to_bf16(f)); }

__global__ __launch_bounds__(256) void k_mlp_to_bf16(const float* __restrict__ theta, uint16_t* __restrict__ out) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < (uint32_t)kParams) out[i] = to_bf16(theta[i]);
}

__global__ __launch_bounds__(256) void k_mlp_infer_bf16(const uint16_t* __restrict__ th, const float* __restrict__ X,
                                                        uint64_t n, float* __restrict__ logits,
                                                        int32_t* __restrict__ pad_choice,
                                                        int32_t* __restrict__ bsz_choice) {
    __shared__ float W[kParams];
    for (int i = threadIdx.x; i < kParams; i += 256) W[i] = from_bf16(th[i]);
    __syncthreads();
    const uint64_t s = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (s >= n) return;
    float xin[kFeat], h1[kHid], h2[kHid];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) xin[k] = round_bf16(X[s * kFeat + k]);
    for (int j = 0; j < kHid; ++j) {
        float acc = W[oB1 + j];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) acc += W[oW1 + j * kFeat + k] * xin[k];
        h1[j] = round_bf16(acc > 0.0f ? acc : 0.0f);
    }
    for (int j = 0; j < kHid; ++j) {
        float acc = W[oB2 + j];
#pragma unroll
        for (int k = 0; k < kHid; ++k) acc += W[oW2 + j * kHid + k] * h1[k];
        h2[j] = round_bf16(acc > 0.0f ? acc : 0.0f);
    }
    float z[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
        float acc = W[oB3 + o];
#pragma unroll
        for (int k = 0; k < kHid; ++k) acc += W[oW3 + o * kHid + k] * h2[k];
        z[o] = acc;
        if (logits) logits[s * kOut + o] = acc;
    }
    int bp = 0, bb = 0;
#pragma unroll
    for (int o = 1; o < kNPad; ++o) bp = z[o] > z[bp] ? o : bp;
#pragma unroll
    for (int o = 1; o < kNBsz; ++o) bb = z[kNPad + o] > z[kNPad + bb] ? o : bb;
    if (pad_choice) pad_choice[s] = bp;
    if (bsz_choice) bsz_choice[s] = bb;
}

dq_status launched() { return hipGetLastError() == hipSuccess ? DQ_OK : DQ_EDEVICE; }

uint64_t mlp_tiles(uint64_t n) { return (n + kTile - 1) / kTile; }
uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

}  // namespace
}  // namespace dq

using namespace dq;

extern "C" {

dq_status dq_block_stats(const dq_params* p, double eb_abs, const float* x, const uint16_t* codes,
                         dq_block_stat* stats, int32_t* status, void* hip_stream) {
    SelGeom g;
    if (!make_sel_geom(p, g) || !x || !stats) return DQ_EINVAL;
    if (!(eb_abs > 0.0) || !std::isfinite(eb_abs) || !std::isfinite(1.0 / (2.0 * eb_abs))) return DQ_EINVAL;
    double cells = 1.0;
    for (int a = 0; a < p->ndim; ++a) cells *= (double)p->block;
    if (cells > 4096.0) return DQ_ENOTSUP;
    const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const uint64_t grid = (g.nblocks + 3) / 4;
    hipLaunchKernelGGL(k_block_stats, dim3((uint32_t)grid), dim3(256), 0, st, g, x, codes, 1.0 / (2.0 * eb_abs),
                       2.0 * eb_abs, eb_abs, stats, status);
    return launched();
}

dq_status dq_block_select(const dq_params* p, const dq_block_stat* stats, int32_t* cand, uint8_t* flags,
                          int32_t* label, float* feat, void* ws, void* hip_stream) {
    SelGeom g;
    if (!make_sel_geom(p, g) || !stats || !cand || !ws) return DQ_EINVAL;
    if ((reinterpret_cast<uintptr_t>(ws) % 8) != 0) return DQ_EINVAL;
    if (p->radius < 1 || p->radius > 32768) return DQ_EINVAL;
    const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    long long* gsum = static_cast<long long*>(ws);
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(64), 0, st, gsum);
    uint64_t gb = (g.nblocks + 255) / 256;
    if (gb > 1024) gb = 1024;
    hipLaunchKernelGGL(k_sum_blocks, dim3((uint32_t)gb), dim3(256), 0, st, stats, g.nblocks, gsum);
    hipLaunchKernelGGL(k_block_select, dim3((uint32_t)((g.nblocks + 255) / 256)), dim3(256), 0, st, g, stats,
                       (const long long*)gsum, (int32_t)p->radius, cand, flags, label, feat);
    return launched();
}

dq_status dq_num_super(const dq_params* p, uint64_t* n_super) {
    SelGeom g;
    if (!make_sel_geom(p, g) || !n_super) return DQ_EINVAL;
    *n_super = (uint64_t)g.nsb[0] * g.nsb[1] * g.nsb[2];
    return DQ_OK;
}

dq_status dq_super_cost(const dq_params* p, const dq_block_stat* stats, const uint8_t* flags,
                        const int32_t* choice, uint64_t* cost, void* hip_stream) {
    SelGeom g;
    if (!make_sel_geom(p, g) || !stats || !flags || !choice || !cost) return DQ_EINVAL;
    hipLaunchKernelGGL(k_super_cost, dim3((uint32_t)((g.nblocks + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), g, stats, flags, choice,
                       reinterpret_cast<unsigned long long*>(cost));
    return launched();
}

dq_status dq_gather_pads(const int32_t* cand, const int32_t* choice, uint64_t n_blocks, int32_t* pads,
                         void* hip_stream) {
    if (!cand || !choice || !pads) return DQ_EINVAL;
    if (n_blocks == 0) return DQ_OK;
    hipLaunchKernelGGL(k_gather_pads, dim3((uint32_t)((n_blocks + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), cand, choice, n_blocks, pads);
    return launched();
}

dq_status dq_mlp_workspace(uint64_t n, uint64_t* bytes) {
    if (!bytes || n == 0) return DQ_EINVAL;
    const uint64_t tiles = mlp_tiles(n);
    *bytes = align256(tiles * kParams * sizeof(float)) + align256(tiles * sizeof(float));
    return DQ_OK;
}

dq_status dq_mlp_grad(const float* theta, const float* X, const int32_t* y_pad, const int32_t* y_bsz, uint64_t n,
                      float* grad, float* loss, void* ws, uint64_t ws_bytes, void* hip_stream) {
    if (!theta || !X || !y_pad || !y_bsz || !grad || !ws || n == 0) return DQ_EINVAL;
    uint64_t need = 0;
    dq_mlp_workspace(n, &need);
    if (ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % 16) != 0) return DQ_EINVAL;
    const uint64_t tiles = mlp_tiles(n);
    if (tiles > 0x7fffffffull) return DQ_EINVAL;
    float* partial = static_cast<float*>(ws);
    float* lossp = reinterpret_cast<float*>(static_cast<char*>(ws) + align256(tiles * kParams * sizeof(float)));
    const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_mlp_tile, dim3((uint32_t)tiles), dim3(256), 0, st, theta, X, y_pad, y_bsz, n, partial, lossp);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, (const float*)partial,
                       (const float*)lossp, (uint32_t)tiles, grad, loss);
    return launched();
}

dq_status dq_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t t, float lr, void* hip_stream) {
    if (!theta || !m || !v || !grad || t < 1) return DQ_EINVAL;
    const float c1 = (float)(1.0 - pow(0.9, (double)t));
    const float c2 = (float)(1.0 - pow(0.999, (double)t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), theta, m, v, grad, lr, c1, c2);
    return launched();
}

dq_status dq_mlp_to_bf16(const float* theta, uint16_t* theta_bf16, void* hip_stream) {
    if (!theta || !theta_bf16) return DQ_EINVAL;
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kParams + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), theta, theta_bf16);
    return launched();
}

dq_status dq_mlp_infer_bf16(const uint16_t* theta_bf16, const float* X, uint64_t n, float* logits,
                            int32_t* pad_choice, int32_t* bsz_choice, void* hip_stream) {
    if (!theta_bf16 || !X) return DQ_EINVAL;
    if (n == 0) return DQ_OK;
    const uint64_t grid = (n + 255) / 256;
    if (grid > 0x7fffffffull) return DQ_EINVAL;
    hipLaunchKernelGGL(k_mlp_infer_bf16, dim3((uint32_t)grid), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), theta_bf16, X, n, logits, pad_choice, bsz_choice);
    return launched();
}

}  // extern "C"
