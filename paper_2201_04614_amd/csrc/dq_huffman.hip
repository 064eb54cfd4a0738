// dq_huffman.hip - canonical Huffman coding of the quantisation codes (gfx950).
//
//  k_huff_hist        histogram (LDS-private bins up to 8192 symbols)
//  k_huff_build       one workgroup: present symbols, bitonic sort by
//                     (frequency, symbol) in LDS, the two-queue construction
//                     and depths (one thread, at most 2048 leaves), the length
//                     limit, canonical codewords
//  k_huff_chunk_words one wave per chunk: bits -> words of every chunk
//  k_huff_scan_*      word offsets of the chunks (two-level scan)
//  k_huff_encode      one wave per chunk: codewords OR-ed into an LDS word
//                     buffer at their bit offsets, then copied out
//  k_huff_dtable      decode tables: counts / first codewords / first ranks per
//                     length, symbols in (length, symbol) order, an 11-bit
//                     lookup table
//  k_huff_decode      four threads per chunk (from its sub-chunk offsets):
//                     64-bit bit buffer in registers,
//                     lookup table for codewords of at most 11 bits, canonical
//                     search above
#include "dq_device.hpp"
#include "dq_huffman.h"

namespace dq {
namespace {

constexpr uint32_t kChunk = DQ_HUFF_CHUNK;
constexpr uint32_t kSub = DQ_HUFF_SUB;  // a chunk is decoded from kChunk / kSub places
constexpr uint32_t kMaxPresent = DQ_HUFF_MAX_PRESENT;
constexpr int kMaxLen = 32;
constexpr int kLutBits = 11;
constexpr uint32_t kLocalBins = 8192;
constexpr uint32_t kStage = 16;              // words a decoding thread stages at a time
constexpr uint64_t kStageMinThreads = 262144;  // staging pays once the decoding threads fill the GPU
constexpr int ST_ENOTSUP = DQ_ENOTSUP;

struct DTable {
    uint32_t count[kMaxLen + 1];
    uint32_t first_code[kMaxLen + 1];
    uint32_t first_index[kMaxLen + 1];
    uint32_t n_present;
    uint32_t lut[1u << kLutBits];  // (symbol << 8) | length, 0 = longer than kLutBits
    uint16_t sorted[kMaxPresent];  // symbols in (length, symbol) order
};

__device__ __forceinline__ void set_status(int32_t* st, int v) {
    // the first error of the call wins
    int expected = ST_OK;
    __hip_atomic_compare_exchange_strong(st, &expected, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_huff_status_ok(int32_t* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *st = ST_OK;
}

__global__ __launch_bounds__(256) void k_huff_zero(uint32_t* p, uint32_t n) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Codes are mostly in a few bins (the residuals of smooth data cluster at
// the centre): alphabets of at most 2048 symbols get one LDS copy of the bins
// per wave, larger ones up to kLocalBins one copy per workgroup, beyond that
// global atomics. vec8: codes are 16-byte aligned, read 8 at a time.
__global__ __launch_bounds__(256) void k_huff_hist(const uint16_t* __restrict__ codes, uint64_t n, uint32_t K,
                                                   int vec8, uint32_t* __restrict__ hist, int32_t* status) {
    __shared__ uint32_t lh[kLocalBins];
    const bool local = K <= kLocalBins;  // uniform
    const uint32_t copies = K <= kLocalBins / 4 ? 4u : 1u;
    uint32_t* mine = lh + (copies == 4u ? (threadIdx.x >> 6) * K : 0u);
    if (local) {
        for (uint32_t s = threadIdx.x; s < copies * K; s += 256u) lh[s] = 0u;
        __syncthreads();
    }
    bool bad = false;
    auto count = [&](uint32_t c) {
        if (c >= K) {
            bad = true;
        } else if (local) {
            atomicAdd(&mine[c], 1u);
        } else {
            atomicAdd(&hist[c], 1u);
        }
    };
    const uint64_t tid = (uint64_t)blockIdx.x * 256u + threadIdx.x, stride = (uint64_t)gridDim.x * 256u;
    uint64_t done = 0;
    if (vec8) {
        const uint4* c8 = reinterpret_cast<const uint4*>(codes);
        const uint64_t n8 = n / 8;
        for (uint64_t i = tid; i < n8; i += stride) {
            const uint4 v = c8[i];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                count(w[k] & 0xffffu);
                count(w[k] >> 16);
            }
        }
        done = n8 * 8;
    }
    for (uint64_t i = done + tid; i < n; i += stride) count(codes[i]);
    if (local) {
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < K; s += 256u) {
            uint32_t v = 0;
            for (uint32_t c = 0; c < copies; ++c) v += lh[c * K + s];
            if (v) atomicAdd(&hist[s], v);
        }
    }
    if (bad) set_status(status, ST_EINVAL);
}

// Present symbols (hist > 0) in symbol order into psym; returns their number
// (the same in every thread). Block of 1024 threads.
__device__ uint32_t compact_present(const uint32_t* __restrict__ hist, uint32_t K, uint16_t* psym,
                                    uint32_t* wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t total = 0;
    for (uint32_t base = 0; base < K; base += 1024u) {
        const uint32_t s = base + (uint32_t)tid;
        const uint32_t p = (s < K && hist[s] > 0u) ? 1u : 0u;
        const uint32_t incl = wave_scan_incl(p, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < 16; ++w) {
            all += wsum[w];
            before += w < wave ? wsum[w] : 0u;
        }
        const uint32_t pos = total + before + incl - p;
        if (p && pos < kMaxPresent) psym[pos] = (uint16_t)s;
        total += all;
        __syncthreads();
    }
    return total;
}

// Ascending bitonic sort of keys[0 .. P) in LDS (P a power of two), by a
// workgroup of 1024 threads.
__device__ void bitonic_sort_lds(unsigned long long* keys, uint32_t P) {
    const uint32_t tid = threadIdx.x;
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < P; i += 1024u) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const unsigned long long a = keys[i], b = keys[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        keys[i] = b;
                        keys[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Canonical order of the n present symbols psym[i] with lengths len[i]
// (both in LDS): keys sorted by (length, symbol), the count of each length,
// its first codeword and its first sorted position. Lengths above kMaxLen
// sort last and are not counted (bad = 1). Workgroup of 1024 threads.
__device__ void canonical_order(const uint8_t* len, const uint16_t* psym, uint32_t n, unsigned long long* keys,
                                uint32_t* cnt, uint32_t* fcode, uint32_t* fidx, int* bad) {
    const uint32_t tid = threadIdx.x;
    if (tid <= (uint32_t)kMaxLen) cnt[tid] = 0u;
    __syncthreads();
    uint32_t P = 1;
    while (P < n) P <<= 1;
    for (uint32_t i = tid; i < P; i += 1024u) {
        if (i < n) {
            const uint32_t l = len[i];
            keys[i] = ((unsigned long long)l << 16) | psym[i];
            if (l > (uint32_t)kMaxLen) *bad = 1;
            else atomicAdd(&cnt[l], 1u);
        } else {
            keys[i] = ~0ull;
        }
    }
    __syncthreads();
    bitonic_sort_lds(keys, P);
    if (tid == 0) {
        unsigned long long code = 0;
        uint32_t idx = 0;
        for (int l = 0; l <= kMaxLen; ++l) {
            if (l > 0) code = (code + (l > 1 ? cnt[l - 1] : 0u)) << 1;
            fcode[l] = (uint32_t)code;
            fidx[l] = idx;
            idx += l > 0 ? cnt[l] : 0u;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_huff_build(const uint32_t* __restrict__ hist, uint32_t K,
                                                     uint8_t* __restrict__ lengths,
                                                     uint32_t* __restrict__ codewords, int32_t* status) {
    __shared__ uint16_t psym[kMaxPresent];
    __shared__ unsigned long long key[kMaxPresent];
    __shared__ unsigned long long wint[kMaxPresent];  // internal weights, then depths
    __shared__ int16_t par_leaf[kMaxPresent], par_int[kMaxPresent];
    __shared__ uint8_t len_sorted[kMaxPresent], len_sym[kMaxPresent];  // by sorted position / by psym position
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t cnt[kMaxLen + 1], fcode[kMaxLen + 1], fidx[kMaxLen + 1];
    __shared__ int too_long, bad;
    const int tid = threadIdx.x;
    for (uint32_t s = tid; s < K; s += 1024u) {
        lengths[s] = 0;
        codewords[s] = 0u;
    }
    const uint32_t np = compact_present(hist, K, psym, wsum);
    if (np > kMaxPresent) {
        if (tid == 0) set_status(status, ST_ENOTSUP);
        return;
    }
    if (np == 0) return;
    __syncthreads();  // lengths / codewords zeroed before they are written below
    if (np == 1) {
        if (tid == 0) {
            lengths[psym[0]] = 1;
            codewords[psym[0]] = 0u;
        }
        return;
    }
    uint32_t P = 1;
    while (P < np) P <<= 1;
    for (int shift = 0; shift < 64; ++shift) {
        // leaves sorted by (frequency, symbol); frequencies halved `shift` times (kept >= 1)
        for (uint32_t i = tid; i < P; i += 1024u) {
            if (i < np) {
                const uint32_t s = psym[i];
                unsigned long long f = (unsigned long long)hist[s] >> shift;
                f = f ? f : 1ull;
                key[i] = (f << 16) | s;
            } else {
                key[i] = ~0ull;
            }
        }
        __syncthreads();
        bitonic_sort_lds(key, P);
        if (tid == 0) {
            // two queues: leaves in key order, internal nodes in creation order;
            // the lighter front first, a leaf on equal weights
            uint32_t li = 0, ji = 0;
            for (uint32_t m = 0; m + 1 < np; ++m) {
                unsigned long long w = 0;
                for (int take = 0; take < 2; ++take) {
                    if (li < np && (ji >= m || (key[li] >> 16) <= wint[ji])) {
                        w += key[li] >> 16;
                        par_leaf[li++] = (int16_t)m;
                    } else {
                        w += wint[ji];
                        par_int[ji++] = (int16_t)m;
                    }
                }
                wint[m] = w;
            }
            // depths: the root is the last internal node; parents come later
            wint[np - 2] = 0;
            for (int j = (int)np - 3; j >= 0; --j) wint[j] = wint[par_int[j]] + 1;
            int longest = 0;
            for (uint32_t i = 0; i < np; ++i) {
                const int L = (int)wint[par_leaf[i]] + 1;
                longest = L > longest ? L : longest;
            }
            too_long = longest > kMaxLen;
        }
        __syncthreads();
        if (!too_long) break;
        __syncthreads();
    }
    for (uint32_t i = tid; i < np; i += 1024u) len_sorted[i] = (uint8_t)(wint[par_leaf[i]] + 1);
    __syncthreads();
    // lengths by symbol: out to memory, and in LDS by the symbol's place in psym
    // (psym is in symbol order: a binary search finds it)
    for (uint32_t i = tid; i < np; i += 1024u) {
        const uint32_t s = (uint32_t)(key[i] & 0xffffu);
        lengths[s] = len_sorted[i];
        uint32_t lo = 0, hi = np;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (psym[mid] < s) lo = mid + 1;
            else hi = mid;
        }
        len_sym[lo] = len_sorted[i];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    // canonical codewords: symbols in (length, symbol) order get consecutive
    // codewords from their length's first one
    canonical_order(len_sym, psym, np, key, cnt, fcode, fidx, &bad);
    for (uint32_t j = tid; j < np; j += 1024u) {
        const uint32_t l = (uint32_t)(key[j] >> 16);
        codewords[key[j] & 0xffffu] = fcode[l] + (j - fidx[l]);
    }
}

__global__ __launch_bounds__(256) void k_huff_chunk_words(const uint16_t* __restrict__ codes, uint64_t n, uint32_t K,
                                                          const uint8_t* __restrict__ lengths,
                                                          uint32_t* __restrict__ chunk_words, int32_t* status) {
    const int lane = threadIdx.x & 63;
    const uint64_t c = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint64_t nch = (n + kChunk - 1) / kChunk;
    if (c >= nch) return;
    const uint64_t base = c * kChunk;
    uint32_t bits = 0;
    bool bad = false;
    for (uint32_t k = 0; k < kChunk / 64; ++k) {
        const uint64_t i = base + (uint64_t)lane * (kChunk / 64) + k;
        if (i < n) {
            const uint32_t s = codes[i];
            const uint32_t L = s < K ? min((uint32_t)lengths[s], (uint32_t)kMaxLen) : 0u;
            bad = bad || L == 0u;
            bits += L;
        }
    }
    bits = (uint32_t)group_sum64<64>((long long)bits);
    if (lane == 0) chunk_words[c] = (bits + 31u) / 32u;
    if (ballot(bad) && lane == 0) set_status(status, ST_EINVAL);
}

// Exclusive scan of n uint32 into n + 1 uint64 (out[n] = total): per 1024
// block, then the block totals (one workgroup), then the carries.
__global__ __launch_bounds__(1024) void k_huff_scan_a(const uint32_t* __restrict__ in, uint64_t n,
                                                      unsigned long long* __restrict__ out,
                                                      unsigned long long* __restrict__ tot) {
    __shared__ unsigned long long ws[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t i = (uint64_t)blockIdx.x * 1024u + tid;
    const unsigned long long v = i < n ? in[i] : 0ull;
    unsigned long long x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    unsigned long long before = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
        all += ws[w];
        before += w < wave ? ws[w] : 0ull;
    }
    if (i < n) out[i] = before + x - v;
    if (tid == 0) tot[blockIdx.x] = all;
}

__global__ __launch_bounds__(1024) void k_huff_scan_b(unsigned long long* __restrict__ tot, uint32_t nb) {
    __shared__ unsigned long long ws[16];
    __shared__ unsigned long long carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base <= nb; base += 1024u) {  // entry nb receives the grand total
        const uint32_t i = base + tid;
        const unsigned long long v = i < nb ? tot[i] : 0ull;
        unsigned long long x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long t = __shfl_up(x, off);
            if (lane >= off) x += t;
        }
        if (lane == 63) ws[wave] = x;
        __syncthreads();
        unsigned long long before = 0, all = 0;
        for (int w = 0; w < 16; ++w) {
            all += ws[w];
            before += w < wave ? ws[w] : 0ull;
        }
        const unsigned long long c0 = carry;
        if (i <= nb) tot[i] = c0 + before + x - v;
        __syncthreads();
        if (tid == 0) carry = c0 + all;
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_huff_scan_c(unsigned long long* __restrict__ out, uint64_t n,
                                                      const unsigned long long* __restrict__ tot, uint32_t nb,
                                                      uint64_t cap, int32_t* status) {
    const uint64_t i = (uint64_t)blockIdx.x * 1024u + threadIdx.x;
    if (i < n) out[i] += tot[blockIdx.x];
    if (i == 0) {
        out[n] = tot[nb];
        if (tot[nb] > cap) set_status(status, ST_ECAPACITY);
    }
}

__global__ __launch_bounds__(256) void k_huff_encode(const uint16_t* __restrict__ codes, uint64_t n, uint32_t K,
                                                     const uint8_t* __restrict__ lengths,
                                                     const uint32_t* __restrict__ codewords,
                                                     const unsigned long long* __restrict__ chunk_off,
                                                     uint32_t* __restrict__ words, uint64_t cap,
                                                     uint16_t* __restrict__ sub_off) {
    __shared__ uint32_t buf[4][kChunk];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t c = (uint64_t)blockIdx.x * 4u + wave;
    const uint64_t nch = (n + kChunk - 1) / kChunk;
    if (c >= nch) return;  // wave-uniform; no workgroup barrier below
    const uint64_t w0 = chunk_off[c], w1 = chunk_off[c + 1];
    if (w1 > cap || w1 < w0 || w1 - w0 > kChunk) return;  // capacity error already reported
    const uint32_t nw = (uint32_t)(w1 - w0);
    uint32_t* b = buf[wave];
    for (uint32_t w = lane; w < nw; w += 64) b[w] = 0u;
    const uint64_t base = c * kChunk + (uint64_t)lane * (kChunk / 64);
    uint32_t L[kChunk / 64], C[kChunk / 64];
    uint32_t bits = 0;
#pragma unroll
    for (uint32_t k = 0; k < kChunk / 64; ++k) {
        const uint64_t i = base + k;
        const uint32_t s = i < n ? codes[i] : K;
        const bool ok = s < K;
        L[k] = ok ? min((uint32_t)lengths[s], (uint32_t)kMaxLen) : 0u;
        C[k] = ok ? codewords[s] : 0u;
        bits += L[k];
    }
    const uint32_t incl = wave_scan_incl(bits, lane);
    uint32_t p = incl - bits;
    // lane l holds codes 16 l ..: the bit offsets of codes 256, 512, 768
    const uint32_t s1 = readlane(p, 16), s2 = readlane(p, 32), s3 = readlane(p, 48);
    if (lane == 0) {
        sub_off[c * 3 + 0] = (uint16_t)s1;
        sub_off[c * 3 + 1] = (uint16_t)s2;
        sub_off[c * 3 + 2] = (uint16_t)s3;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (uint32_t k = 0; k < kChunk / 64; ++k) {
        const uint32_t len = L[k];
        if (len) {
            const uint32_t w = p >> 5, avail = 32u - (p & 31u);
            if (len <= avail) {
                atomicOr(&b[w], C[k] << (avail - len));
            } else {
                atomicOr(&b[w], C[k] >> (len - avail));
                atomicOr(&b[w + 1], C[k] << (32u - (len - avail)));
            }
            p += len;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t w = lane; w < nw; w += 64) words[w0 + w] = b[w];
}

__global__ __launch_bounds__(1024) void k_huff_dtable(const uint8_t* __restrict__ lengths, uint32_t K,
                                                      DTable* __restrict__ t, int32_t* status) {
    __shared__ uint16_t psym[kMaxPresent];
    __shared__ uint16_t sorted[kMaxPresent];
    __shared__ uint8_t lenp[kMaxPresent];
    __shared__ unsigned long long keys[kMaxPresent];
    __shared__ uint32_t lut[1u << kLutBits];
    __shared__ uint32_t cnt[kMaxLen + 1], fcode[kMaxLen + 1], fidx[kMaxLen + 1];
    __shared__ uint32_t wsum[16];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // present symbols: lengths > 0 (compaction in symbol order)
    uint32_t total = 0;
    for (uint32_t base = 0; base < K; base += 1024u) {
        const uint32_t s = base + (uint32_t)tid;
        const uint32_t pr = (s < K && lengths[s] > 0) ? 1u : 0u;
        const uint32_t incl = wave_scan_incl(pr, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < 16; ++w) {
            all += wsum[w];
            before += w < wave ? wsum[w] : 0u;
        }
        const uint32_t pos = total + before + incl - pr;
        if (pr && pos < kMaxPresent) psym[pos] = (uint16_t)s;
        total += all;
        __syncthreads();
    }
    if (total > kMaxPresent) {
        for (uint32_t i = tid; i < (1u << kLutBits); i += 1024u) t->lut[i] = 0u;
        if (tid == 0) {
            t->n_present = 0;
            set_status(status, ST_ENOTSUP);
        }
        return;
    }
    for (uint32_t i = tid; i < total; i += 1024u) lenp[i] = lengths[psym[i]];
    for (uint32_t i = tid; i < (1u << kLutBits); i += 1024u) lut[i] = 0u;
    if (tid == 0) bad = 0;
    __syncthreads();
    canonical_order(lenp, psym, total, keys, cnt, fcode, fidx, &bad);
    // symbols in (length, symbol) order, and the lookup table: the codeword at
    // sorted position j (length l <= kLutBits) covers 2^(kLutBits - l)
    // entries; lengths that break the prefix property could reach past it
    for (uint32_t j = tid; j < total; j += 1024u) {
        const uint32_t l = (uint32_t)(keys[j] >> 16);
        const uint32_t sym = (uint32_t)(keys[j] & 0xffffu);
        sorted[j] = (uint16_t)sym;
        if (l > (uint32_t)kLutBits) continue;
        const unsigned long long cw = (unsigned long long)fcode[l] + (j - fidx[l]);
        const unsigned long long lo = cw << (kLutBits - l), hi = (cw + 1ull) << (kLutBits - l);
        if (hi > (1ull << kLutBits)) {
            bad = 1;
            continue;
        }
        for (unsigned long long e = lo; e < hi; ++e) lut[e] = (sym << 8) | l;
    }
    __syncthreads();
    for (uint32_t i = tid; i < (1u << kLutBits); i += 1024u) t->lut[i] = lut[i];
    for (uint32_t i = tid; i < total; i += 1024u) t->sorted[i] = sorted[i];
    if (tid <= kMaxLen) {
        t->count[tid] = cnt[tid];
        t->first_code[tid] = fcode[tid];
        t->first_index[tid] = fidx[tid];
    }
    if (tid == 0) {
        t->n_present = total;
        if (bad) set_status(status, ST_EINVAL);
    }
}

// staged: with many chunks (several waves per CU) every thread loads its
// next kStage words at once into LDS (one latency per ~kStage * 32 bits);
// with few chunks each thread's serial decoding chain dominates, and it
// loads the next word one refill ahead in a register instead.
__global__ __launch_bounds__(256) void k_huff_decode(const uint32_t* __restrict__ words, uint64_t n_words,
                                                     const unsigned long long* __restrict__ chunk_off, uint64_t n,
                                                     const uint16_t* __restrict__ sub_off,
                                                     const DTable* __restrict__ t, uint16_t* __restrict__ out,
                                                     int32_t* status, int staged) {
    __shared__ uint32_t lut[1u << kLutBits];
    __shared__ uint16_t sorted[kMaxPresent];
    __shared__ uint32_t cnt[kMaxLen + 1], fcode[kMaxLen + 1], fidx[kMaxLen + 1];
    __shared__ uint32_t stage[256][kStage + 1];
    for (uint32_t i = threadIdx.x; i < (1u << kLutBits); i += 256u) lut[i] = t->lut[i];
    const uint32_t np = min(t->n_present, kMaxPresent);
    for (uint32_t i = threadIdx.x; i < np; i += 256u) sorted[i] = t->sorted[i];
    if (threadIdx.x <= (uint32_t)kMaxLen) {
        cnt[threadIdx.x] = t->count[threadIdx.x];
        fcode[threadIdx.x] = t->first_code[threadIdx.x];
        fidx[threadIdx.x] = t->first_index[threadIdx.x];
    }
    __syncthreads();
    const uint64_t tg = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t c = tg / (kChunk / kSub);                   // chunk
    const uint32_t part = (uint32_t)(tg % (kChunk / kSub));    // its part
    const uint64_t nch = (n + kChunk - 1) / kChunk;
    if (c >= nch) return;
    const uint32_t mc = (uint32_t)min((uint64_t)kChunk, n - c * kChunk);
    if (part * kSub >= mc) return;
    const uint32_t m = min(kSub, mc - part * kSub);
    const uint64_t wbeg = chunk_off[c];
    const uint64_t wend = min(chunk_off[c + 1], n_words);  // reads stay inside the words buffer
    if (wend < wbeg) {
        set_status(status, ST_ECORRUPT);
        return;
    }
    const uint32_t start = part ? sub_off[c * 3 + part - 1] : 0u;  // bit offset in the chunk
    uint64_t w = wbeg + (start >> 5);
    uint64_t used = start;
    bool bad = false;
    // the first word, its leading bits skipped
    unsigned long long buf = (unsigned long long)(w < wend ? words[w] : 0u) << (32 + (start & 31u));
    int have = 32 - (int)(start & 31u);
    ++w;
    uint16_t* o = out + c * kChunk + part * kSub;
    uint32_t* sb = stage[threadIdx.x];
    uint32_t sidx = kStage;
    uint32_t pre = 0;
    if (!staged) {
        pre = w < wend ? words[w] : 0u;
        ++w;
    }
    for (uint32_t i = 0; i < m; ++i) {
        while (have <= 32) {  // keep at least 33 bits: every codeword fits
            unsigned long long v;
            if (staged) {
                if (sidx == kStage) {  // kStage independent loads, one latency
#pragma unroll
                    for (uint32_t k = 0; k < kStage; ++k) sb[k] = (w + k < wend) ? words[w + k] : 0u;
                    w += kStage;
                    sidx = 0;
                }
                v = sb[sidx++];
            } else {  // the next word was loaded at the previous refill
                v = pre;
                pre = w < wend ? words[w] : 0u;
                ++w;
            }
            buf |= v << (32 - have);
            have += 32;
        }
        const uint32_t e = lut[(uint32_t)(buf >> (64 - kLutBits))];
        uint32_t len = e & 0xffu, sym = e >> 8;
        if (len == 0) {
            for (len = kLutBits + 1; len <= (uint32_t)kMaxLen; ++len) {
                const uint32_t code = (uint32_t)(buf >> (64 - len));
                const uint32_t r = code - fcode[len];
                if (r < cnt[len]) {
                    sym = sorted[min(fidx[len] + r, kMaxPresent - 1)];
                    break;
                }
            }
            if (len > (uint32_t)kMaxLen) {  // does not parse
                bad = true;
                len = 1;
                sym = 0;
            }
        }
        o[i] = (uint16_t)sym;
        buf <<= len;
        have -= (int)len;
        used += len;
    }
    if (bad || used > (wend - wbeg) * 32ull) set_status(status, ST_ECORRUPT);
}

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

struct Layout {
    uint64_t chunk_words, tot, dtable, total;
};

Layout layout(uint64_t n) {
    const uint64_t nch = (n + kChunk - 1) / kChunk;
    const uint64_t nb = (nch + 1023) / 1024;
    Layout L;
    L.chunk_words = 0;
    L.tot = align256(4 * (nch ? nch : 1));
    L.dtable = L.tot + align256(8 * (nb + 1));
    L.total = L.dtable + align256(sizeof(DTable));
    return L;
}

dq_status launched() { return hipGetLastError() == hipSuccess ? DQ_OK : DQ_EDEVICE; }

}  // namespace
}  // namespace dq

using namespace dq;

extern "C" {

dq_status dq_huff_workspace(uint64_t n, uint64_t* bytes) {
    if (!bytes || n == 0 || n > 0xffffffffull) return DQ_EINVAL;
    *bytes = layout(n).total;
    return DQ_OK;
}

dq_status dq_huff_max_words(uint64_t n, uint64_t* words) {
    if (!words || n == 0 || n > 0xffffffffull) return DQ_EINVAL;
    *words = n + (n + kChunk - 1) / kChunk;
    return DQ_OK;
}

dq_status dq_huff_codebook(const uint16_t* codes, uint64_t n, uint32_t n_symbols, uint32_t* hist, uint8_t* lengths,
                           uint32_t* codewords, int32_t* status, void* ws, uint64_t ws_bytes, void* hip_stream) {
    (void)ws;
    (void)ws_bytes;
    if (!codes || !hist || !lengths || !codewords || !status || n == 0 || n > 0xffffffffull) return DQ_EINVAL;
    if (n_symbols < 1 || n_symbols > DQ_HUFF_MAX_SYMBOLS) return DQ_EINVAL;
    const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_huff_status_ok, dim3(1), dim3(64), 0, st, status);
    hipLaunchKernelGGL(k_huff_zero, dim3((n_symbols + 255) / 256), dim3(256), 0, st, hist, n_symbols);
    uint64_t grid = (n + 256 * 16 - 1) / (256 * 16);
    if (grid > 1024) grid = 1024;
    const int vec8 = (reinterpret_cast<uintptr_t>(codes) % 16) == 0 ? 1 : 0;
    hipLaunchKernelGGL(k_huff_hist, dim3((uint32_t)grid), dim3(256), 0, st, codes, n, n_symbols, vec8, hist,
                       status);
    hipLaunchKernelGGL(k_huff_build, dim3(1), dim3(1024), 0, st, (const uint32_t*)hist, n_symbols, lengths,
                       codewords, status);
    return launched();
}

dq_status dq_huff_encode(const uint16_t* codes, uint64_t n, uint32_t n_symbols, const uint8_t* lengths,
                         const uint32_t* codewords, uint64_t* chunk_off, uint16_t* sub_off, uint32_t* words,
                         uint64_t words_cap, int32_t* status, void* ws, uint64_t ws_bytes, void* hip_stream) {
    if (!codes || !lengths || !codewords || !chunk_off || !sub_off || !words || !status || !ws) return DQ_EINVAL;
    if (n == 0 || n > 0xffffffffull || n_symbols < 1 || n_symbols > DQ_HUFF_MAX_SYMBOLS) return DQ_EINVAL;
    const Layout L = layout(n);
    if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) % 256) != 0) return DQ_EINVAL;
    const uint64_t nch = (n + kChunk - 1) / kChunk;
    const uint64_t nb = (nch + 1023) / 1024;
    char* w = static_cast<char*>(ws);
    uint32_t* cw = reinterpret_cast<uint32_t*>(w + L.chunk_words);
    unsigned long long* tot = reinterpret_cast<unsigned long long*>(w + L.tot);
    unsigned long long* off = reinterpret_cast<unsigned long long*>(chunk_off);
    const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_huff_status_ok, dim3(1), dim3(64), 0, st, status);
    hipLaunchKernelGGL(k_huff_chunk_words, dim3((uint32_t)((nch + 3) / 4)), dim3(256), 0, st, codes, n, n_symbols,
                       lengths, cw, status);
    hipLaunchKernelGGL(k_huff_scan_a, dim3((uint32_t)nb), dim3(1024), 0, st, (const uint32_t*)cw, nch, off, tot);
    hipLaunchKernelGGL(k_huff_scan_b, dim3(1), dim3(1024), 0, st, tot, (uint32_t)nb);
    hipLaunchKernelGGL(k_huff_scan_c, dim3((uint32_t)nb), dim3(1024), 0, st, off, nch,
                       (const unsigned long long*)tot, (uint32_t)nb, words_cap, status);
    hipLaunchKernelGGL(k_huff_encode, dim3((uint32_t)((nch + 3) / 4)), dim3(256), 0, st, codes, n, n_symbols,
                       lengths, codewords, (const unsigned long long*)off, words, words_cap, sub_off);
    return launched();
}

dq_status dq_huff_decode(const uint32_t* words, uint64_t n_words, const uint64_t* chunk_off,
                         const uint16_t* sub_off, uint64_t n, uint32_t n_symbols, const uint8_t* lengths,
                         uint16_t* codes, int32_t* status, void* ws, uint64_t ws_bytes, void* hip_stream) {
    if (!words || !chunk_off || !sub_off || !lengths || !codes || !status || !ws) return DQ_EINVAL;
    if (n == 0 || n > 0xffffffffull || n_symbols < 1 || n_symbols > DQ_HUFF_MAX_SYMBOLS) return DQ_EINVAL;
    const Layout L = layout(n);
    if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) % 256) != 0) return DQ_EINVAL;
    const uint64_t nch = (n + kChunk - 1) / kChunk;
    DTable* t = reinterpret_cast<DTable*>(static_cast<char*>(ws) + L.dtable);
    const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_huff_status_ok, dim3(1), dim3(64), 0, st, status);
    hipLaunchKernelGGL(k_huff_dtable, dim3(1), dim3(1024), 0, st, lengths, n_symbols, t, status);
    const uint64_t threads = nch * (kChunk / kSub);
    hipLaunchKernelGGL(k_huff_decode, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, st, words, n_words,
                       reinterpret_cast<const unsigned long long*>(chunk_off), n, sub_off, (const DTable*)t, codes,
                       status, threads >= kStageMinThreads ? 1 : 0);
    return launched();
}

}  // extern "C"
