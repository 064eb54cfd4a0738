// dq_api.hip - host side of libdq: parameter validation, geometry, workspace
// layout and the launch sequence of dq_compress / dq_decompress.
#include <math.h>
#include <string.h>
#include <time.h>
#include <unistd.h>

#include <atomic>
#include <mutex>

#include "../../include/dq.h"
#include "dq_host.hpp"

using namespace dq;
using namespace dq::host;

namespace dq {
namespace host {

int ilog2(uint32_t v) {
    int l = 0;
    while ((1u << l) < v) ++l;
    return l;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Host check shared by every entry point. check_eb is false for decompress,
// which takes the absolute bound separately.
dq_status validate(const dq_params* p, bool check_eb) {
    if (!p) return DQ_EINVAL;
    if (p->ndim < 1 || p->ndim > 3) return DQ_EINVAL;
    double total = 1.0;
    for (int a = 0; a < p->ndim; ++a) {
        if (p->shape[a] < 1) return DQ_EINVAL;
        total *= (double)p->shape[a];
    }
    if (total > 4294967295.0) return DQ_EINVAL;
    if (check_eb) {
        if (!(p->eb > 0.0) || !isfinite(p->eb)) return DQ_EINVAL;
        if (p->eb_mode != DQ_EB_ABS && p->eb_mode != DQ_EB_REL) return DQ_EINVAL;
        if (p->eb_mode == DQ_EB_ABS && !isfinite(1.0 / (2.0 * p->eb))) return DQ_EINVAL;
    }
    if (p->block < 1) return DQ_EINVAL;
    if (p->pad_mode < DQ_PAD_ZERO || p->pad_mode > DQ_PAD_GIVEN) return DQ_EINVAL;
    if (p->radius < 1 || p->radius > 32768) return DQ_EINVAL;
    if (p->vec != 0 && p->vec != 1 && p->vec != 2 && p->vec != 4) return DQ_EINVAL;
    // GPU kernel coverage
    const int maxb = p->ndim == 1 ? 4096 : (p->ndim == 2 ? 256 : 64);
    if (!is_pow2(p->block) || p->block > maxb) return DQ_ENOTSUP;
    // 2-D blocks wider than a wave step of single cells (128, 256) exist
    // only with block / 64 or more cells per lane, whose row starts must be
    // aligned to that width
    if (p->ndim == 2 && p->block > 64 && p->shape[1] % (p->block / 64) != 0) return DQ_ENOTSUP;
    return DQ_OK;
}

void base_geom(const dq_params* p, Geom& g) {
    const int d = p->ndim;
    const uint32_t B = (uint32_t)p->block;
    g.nx = (uint32_t)p->shape[d - 1];
    g.ny = d >= 2 ? (uint32_t)p->shape[d - 2] : 1u;
    g.nz = d == 3 ? (uint32_t)p->shape[0] : 1u;
    g.nbx = (g.nx + B - 1) / B;
    g.nby = (g.ny + B - 1) / B;
    g.nbz = (g.nz + B - 1) / B;
    g.nblocks = g.nbx * g.nby * g.nbz;
    g.N = (uint64_t)g.nx * g.ny * g.nz;
}

bool finish_plan(const dq_params* p, int V, Plan& pl) {
    const int bpt = tile_blocks(p->ndim, p->block, V);
    if (bpt <= 0) return false;
    base_geom(p, pl.g);
    if (pl.g.nx % (uint32_t)V != 0) return false;
    pl.g.bpt = (uint32_t)bpt;
    pl.g.ntx = (pl.g.nbx + (uint32_t)bpt - 1) / (uint32_t)bpt;
    const uint64_t tiles = (uint64_t)pl.g.ntx * pl.g.nby * pl.g.nbz;
    if (tiles > 0xffffffffull) return false;
    pl.g.n_tiles = (uint32_t)tiles;
    pl.dim = p->ndim;
    pl.B = p->block;
    pl.V = V;
    pl.nblocks = pl.g.nblocks;
    return true;
}

// Widest vector width V that the field and the buffers allow.
bool make_plan(const dq_params* p, const void* fptr, const void* cptr, Plan& pl) {
    const uintptr_t fa = reinterpret_cast<uintptr_t>(fptr);
    const uintptr_t ca = reinterpret_cast<uintptr_t>(cptr);
    if (p->vec) {
        const int V = p->vec;
        if ((fa % (4u * V)) == 0 && (ca % (2u * V)) == 0 && finish_plan(p, V, pl)) return true;
    }
    // Automatic: the vector width that keeps the most waves resident on every
    // SIMD, min(encode occupancy, tiles per SIMD); ties go to the wider one
    // (fewer instructions per cell).
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    bool found = false;
    double best = -1.0;
    for (int V = 4; V >= 1; V >>= 1) {
        if ((fa % (4u * V)) != 0 || (ca % (2u * V)) != 0) continue;
        Plan cand;
        if (!finish_plan(p, V, cand)) continue;
        int occ = encode_occupancy(p->ndim, p->block, V);
        if (occ < 1) occ = 1;
        const double per_simd = (double)cand.g.n_tiles / (4.0 * cus);
        const double resident = per_simd < occ ? per_simd : (double)occ;
        if (!found || resident > best) {
            pl = cand;
            best = resident;
            found = true;
        }
    }
    return found;
}

uint64_t max_tiles(const dq_params* p) {
    uint64_t m = 0;
    for (int V = 1; V <= 4; V <<= 1) {
        Plan pl;
        if (finish_plan(p, V, pl) && pl.g.n_tiles > m) m = pl.g.n_tiles;
    }
    return m;
}

CompressLayout compress_layout(const dq_params* p, uint64_t out_cap) {
    Geom g;
    base_geom(p, g);
    const uint64_t cap = out_cap < g.N ? out_cap : g.N;
    const uint64_t mt = max_tiles(p);
    CompressLayout L;
    L.cap = cap;
    L.sc = 0;
    L.parts = align_up(sizeof(Scalars));
    L.tiles = L.parts + align_up(sizeof(uint2) * kMinmaxParts);
    L.toff = L.tiles + align_up(4 * mt);
    L.csum = L.toff + align_up(4 * mt);
    L.info = L.csum + align_up(4 * ((mt + kChunkTiles - 1) / kChunkTiles));
    L.region = L.info + align_up(4ull * g.nblocks);
    L.ovf = L.region + align_up(16 * cap);
    L.total = L.ovf + align_up(16 * (cap > 0 ? cap : 1));
    return L;
}

// Tag of a decompress call (see status_init_tagged): distinct for every call
// of the process, never 0, salted per process so that a result buffer left
// over from another process is unlikely to carry the same tag.
bool codes_rows_on_lines(const Geom& g, int dim, const void* codes) {
    return (reinterpret_cast<uintptr_t>(codes) & 127u) == 0u && (dim == 1 || g.nx % 64u == 0u);
}

uint32_t next_tag() {
    static std::atomic<uint32_t> counter{0};
    static const uint32_t salt = [] {
        const uint64_t t = (uint64_t)time(nullptr) ^ ((uint64_t)getpid() << 20) ^
                           (uint64_t)reinterpret_cast<uintptr_t>(&counter);
        return (uint32_t)(t ^ (t >> 32)) * 2654435761u;
    }();
    uint32_t tag = 0;
    while (tag == 0) tag = (counter.fetch_add(1) + 1) * 2654435761u ^ salt;
    return tag;
}

}  // namespace host
}  // namespace dq

namespace {

dq_status check_launch() {
    return hipGetLastError() == hipSuccess ? DQ_OK : DQ_EDEVICE;
}

}  // namespace

extern "C" {

dq_status dq_validate(const dq_params* p) { return validate(p, true); }

dq_status dq_num_blocks(const dq_params* p, uint64_t* n_blocks) {
    dq_status st = validate(p, false);
    if (st != DQ_OK && st != DQ_ENOTSUP) return st;
    if (!n_blocks) return DQ_EINVAL;
    uint64_t nb = 1;
    for (int a = 0; a < p->ndim; ++a) nb *= (uint64_t)((p->shape[a] + p->block - 1) / p->block);
    *n_blocks = nb;
    return DQ_OK;
}

dq_status dq_pad_count(const dq_params* p, uint64_t* n_pads) {
    uint64_t nb = 0;
    dq_status st = dq_num_blocks(p, &nb);
    if (st != DQ_OK) return st;
    if (!n_pads) return DQ_EINVAL;
    switch (p->pad_mode) {
    case DQ_PAD_ZERO: *n_pads = 0; break;
    case DQ_PAD_GLOBAL_MEAN:
    case DQ_PAD_GLOBAL_MIN:
    case DQ_PAD_GLOBAL_MAX: *n_pads = 1; break;
    case DQ_PAD_BLOCK_MEAN:
    case DQ_PAD_BLOCK_MIN:
    case DQ_PAD_BLOCK_MAX:
    case DQ_PAD_GIVEN: *n_pads = nb; break;
    default: *n_pads = nb * (uint64_t)p->ndim; break;
    }
    return DQ_OK;
}

dq_status dq_compress_workspace(const dq_params* p, uint64_t out_cap, uint64_t* bytes) {
    dq_status st = validate(p, true);
    if (st != DQ_OK) return st;
    if (!bytes) return DQ_EINVAL;
    *bytes = compress_layout(p, out_cap).total;
    return DQ_OK;
}

dq_status dq_decompress_workspace(const dq_params* p, uint64_t* bytes) {
    dq_status st = validate(p, false);
    if (st != DQ_OK) return st;
    if (!bytes) return DQ_EINVAL;
    Geom g;
    base_geom(p, g);
    *bytes = align_up(4ull * ((uint64_t)g.nblocks + 1));
    return DQ_OK;
}

}  // extern "C"

namespace {

// Host checks of dq_compress and dq_compress_noalloc that need no workspace.
dq_status compress_check(const dq_params* p, const float* x, uint16_t* codes, uint32_t* out_idx,
                         int32_t* out_val, uint64_t out_cap, int32_t* pads, dq_result* res) {
    dq_status st = validate(p, true);
    if (st != DQ_OK) return st;
    uint64_t npads = 0;
    dq_pad_count(p, &npads);
    if (!x || !codes || !res) return DQ_EINVAL;
    if ((reinterpret_cast<uintptr_t>(res) % 8) != 0) return DQ_EINVAL;
    if (out_cap > 0 && (!out_idx || !out_val)) return DQ_EINVAL;
    if (npads > 0 && !pads) return DQ_EINVAL;
    return DQ_OK;
}

// The launch sequence of a compress call over the workspace ws (checked by
// compress_check first).
dq_status compress_impl(const dq_params* p, const float* x, uint16_t* codes, uint32_t* out_idx,
                        int32_t* out_val, uint64_t out_cap, int32_t* pads, dq_result* res, void* ws,
                        uint64_t ws_bytes, void* hip_stream, const dq_hooks* hooks) {
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return DQ_EINVAL;
    Plan pl;
    if (!make_plan(p, x, codes, pl)) return DQ_ENOTSUP;
    const CompressLayout L = compress_layout(p, out_cap);
    if (ws_bytes < L.total) return DQ_EINVAL;
    const uint64_t cap = out_cap < pl.g.N ? out_cap : pl.g.N;

    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    char* w = static_cast<char*>(ws);
    Scalars* sc = reinterpret_cast<Scalars*>(w + L.sc);
    uint32_t* tiles = reinterpret_cast<uint32_t*>(w + L.tiles);
    uint32_t* toff = reinterpret_cast<uint32_t*>(w + L.toff);
    uint32_t* info = reinterpret_cast<uint32_t*>(w + L.info);
    Staging stg;
    stg.spt = (uint32_t)(cap / pl.g.n_tiles);
    stg.region = reinterpret_cast<uint4*>(w + L.region);
    stg.ovf = reinterpret_cast<uint4*>(w + L.ovf);
    stg.ovf_cap = (uint32_t)cap;
    stg.bcells = (uint32_t)pl.B * (pl.dim >= 2 ? (uint32_t)pl.B : 1u) * (pl.dim == 3 ? (uint32_t)pl.B : 1u);
    // a tile holds at most min(bpt, nbx) blocks
    const uint64_t tile_blocks_max = pl.g.bpt < pl.g.nbx ? pl.g.bpt : pl.g.nbx;
    stg.dense = (stg.spt > 0 && tile_blocks_max * stg.bcells <= 2ull * stg.spt) ? 1u : 0u;
    int32_t* status = &res->status;

    uint2* parts = reinterpret_cast<uint2*>(w + L.parts);
    AuxArgs aa{x, sc, status, pl.g.N};
    // parts: read but unused without the value-range pass
    BoundArgs bound{parts, 0, p->eb, p->eb_mode == DQ_EB_REL ? 1 : 0};
    const bool extreme = p->pad_mode == DQ_PAD_GLOBAL_MIN || p->pad_mode == DQ_PAD_GLOBAL_MAX;
    if (p->eb_mode == DQ_EB_REL || extreme) {
        bound.nparts = launch_minmax(aa, parts, res, stream);  // also initialises the call
    } else {
        launch_compress_init(sc, res, p->eb, stream);
    }
    if (p->pad_mode == DQ_PAD_GLOBAL_MEAN) launch_sumq(aa, bound, stream);

    EncArgs ea;
    ea.bound = bound;
    ea.eb_out = &res->eb_abs;
    ea.x = x;
    ea.codes = codes;
    ea.pads = pads;
    ea.block_info = info;
    ea.tile_count = tiles;
    ea.stg = stg;
    ea.sc = sc;
    ea.status = status;
    ea.g = pl.g;
    ea.R = p->radius;
    ea.pad_mode = p->pad_mode;
    const dim3 grid((pl.g.n_tiles + kWaves - 1) / kWaves);
    if (hooks && hooks->ev_before) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(hooks->ev_before), stream);
    if (!launch_encode(pl.dim, pl.B, pl.V, ea, grid, stream)) return DQ_ENOTSUP;
    if (hooks && hooks->ev_after) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(hooks->ev_after), stream);
    if (pl.g.n_tiles <= kPlaceTiles) {
        launch_place(stg, sc, res, out_cap, tiles, pl.g.n_tiles, info, pl.g, out_idx, out_val, stream);
    } else {
        uint32_t* csum = reinterpret_cast<uint32_t*>(w + L.csum);
        launch_chunked_place(stg, sc, res, out_cap, tiles, toff, csum, pl.g.n_tiles, info, pl.g, out_idx, out_val,
                             stream);
    }
    return check_launch();
}

// Workspace of dq_compress_noalloc: one array per device, in the code object
// (no allocation call ever makes it), kept until the process ends. Host code
// never passes the array's name to a kernel (on the host it only stands for
// the symbol): the device address of each device's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
__device__ __align__(256) char scratch[DQ_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

dq_status scratch_of_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DQ_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DQ_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DQ_OK;
}

}  // namespace

extern "C" {

dq_status dq_compress(const dq_params* p, const float* x, uint16_t* codes, uint32_t* out_idx,
                      int32_t* out_val, uint64_t out_cap, int32_t* pads, dq_result* res, void* ws,
                      uint64_t ws_bytes, void* hip_stream, const dq_hooks* hooks) {
    const dq_status st = compress_check(p, x, codes, out_idx, out_val, out_cap, pads, res);
    if (st != DQ_OK) return st;
    return compress_impl(p, x, codes, out_idx, out_val, out_cap, pads, res, ws, ws_bytes, hip_stream, hooks);
}

dq_status dq_compress_noalloc(const dq_params* p, const float* x, uint16_t* codes, uint32_t* out_idx,
                              int32_t* out_val, uint64_t out_cap, int32_t* pads, dq_result* res,
                              void* hip_stream) {
    const dq_status st = compress_check(p, x, codes, out_idx, out_val, out_cap, pads, res);
    if (st != DQ_OK) return st;
    // the size check needs no GPU: a call that cannot fit is refused first
    if (compress_layout(p, out_cap).total > (uint64_t)DQ_SCRATCH_BYTES) return DQ_ENOSCRATCH;
    void* ws = nullptr;
    const dq_status sst = scratch_of_current_device(&ws);
    if (sst != DQ_OK) return sst;
    // every kernel of the sequence initialises the workspace words it reads
    // (the call's scalars and counters are written by its first kernel), so
    // the contents left by an earlier call need no clearing
    return compress_impl(p, x, codes, out_idx, out_val, out_cap, pads, res, ws, DQ_SCRATCH_BYTES, hip_stream,
                         nullptr);
}

}  // extern "C"

namespace {

// Shared by dq_decompress (host count and bound) and dq_decompress_dev (both
// read on the device from the compress result src; cap = its capacity).
dq_status decompress_impl(const dq_params* p, double eb_abs, uint64_t n_out, const dq_result* src, uint64_t cap,
                          const uint16_t* codes, const uint32_t* out_idx, const int32_t* out_val,
                          const int32_t* pads, float* x_hat, dq_result* res, void* ws, uint64_t ws_bytes,
                          void* hip_stream, const dq_hooks* hooks) {
    dq_status st = validate(p, false);
    if (st != DQ_OK) return st;
    if (!src && (!(eb_abs > 0.0) || !isfinite(eb_abs))) return DQ_EINVAL;
    uint64_t npads = 0;
    dq_pad_count(p, &npads);
    if (!codes || !x_hat || !res) return DQ_EINVAL;
    if ((reinterpret_cast<uintptr_t>(res) % 8) != 0) return DQ_EINVAL;  // one 64-bit status word
    if (src && (reinterpret_cast<uintptr_t>(src) % 8) != 0) return DQ_EINVAL;
    const uint64_t most = src ? cap : n_out;  // the largest count the kernels may see
    if (most > 0 && (!out_idx || !out_val || !ws)) return DQ_EINVAL;
    if (npads > 0 && !pads) return DQ_EINVAL;
    Plan pl;
    if (!make_plan(p, x_hat, codes, pl)) return DQ_ENOTSUP;
    if (n_out > pl.g.N) return DQ_EINVAL;
    const uint64_t capn = cap < pl.g.N ? cap : pl.g.N;
    uint64_t need = 0;
    dq_decompress_workspace(p, &need);
    if (most > 0 && ws_bytes < need) return DQ_EINVAL;

    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    uint32_t* block_start = static_cast<uint32_t*>(ws);
    const uint32_t tag = next_tag();
    if (src) launch_result_reset(res, stream);
    if (src ? capn > 0 : n_out > 0)
        launch_index(out_idx, (uint32_t)n_out, pl.g, ilog2((uint32_t)pl.B), pl.dim, block_start, res, tag, stream,
                     src, (uint32_t)capn);

    DecArgs da;
    da.src = reinterpret_cast<const ResultView*>(src);
    da.cap = (uint32_t)capn;
    da.res_word = reinterpret_cast<unsigned long long*>(res);
    da.n_out_out = reinterpret_cast<unsigned long long*>(&res->n_out);
    da.eb_out = &res->eb_abs;
    da.eb_abs = src ? 1.0 : eb_abs;
    da.tag = tag;
    da.codes = codes;
    da.out_idx = out_idx;
    da.out_val = out_val;
    da.pads = pads;
    da.block_start = block_start;
    da.x_hat = x_hat;
    da.g = pl.g;
    da.twoeb = 2.0 * da.eb_abs;
    da.n_out = (uint32_t)n_out;
    da.R = p->radius;
    da.pad_mode = p->pad_mode;
    const dim3 grid((pl.g.n_tiles + kWaves - 1) / kWaves);
    if (hooks && hooks->ev_before) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(hooks->ev_before), stream);
    if (!launch_decode(pl.dim, pl.B, pl.V, da, grid, stream, codes_rows_on_lines(pl.g, pl.dim, codes)))
        return DQ_ENOTSUP;
    if (hooks && hooks->ev_after) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(hooks->ev_after), stream);
    return check_launch();
}

}  // namespace

extern "C" {

dq_status dq_decompress(const dq_params* p, double eb_abs, const uint16_t* codes, const uint32_t* out_idx,
                        const int32_t* out_val, uint64_t n_out, const int32_t* pads, float* x_hat,
                        dq_result* res, void* ws, uint64_t ws_bytes, void* hip_stream,
                        const dq_hooks* hooks) {
    return decompress_impl(p, eb_abs, n_out, nullptr, 0, codes, out_idx, out_val, pads, x_hat, res, ws, ws_bytes,
                           hip_stream, hooks);
}

dq_status dq_decompress_dev(const dq_params* p, const dq_result* cres, uint64_t out_cap, const uint16_t* codes,
                            const uint32_t* out_idx, const int32_t* out_val, const int32_t* pads, float* x_hat,
                            dq_result* res, void* ws, uint64_t ws_bytes, void* hip_stream, const dq_hooks* hooks) {
    if (!cres) return DQ_EINVAL;
    return decompress_impl(p, 0.0, 0, cres, out_cap, codes, out_idx, out_val, pads, x_hat, res, ws, ws_bytes,
                           hip_stream, hooks);
}

dq_status dq_result_sync(const dq_result* res_dev, dq_result* res_host, void* hip_stream) {
    if (!res_dev || !res_host) return DQ_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipMemcpyAsync(res_host, res_dev, sizeof(dq_result), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return DQ_EDEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return DQ_EDEVICE;
    return DQ_OK;
}

dq_status dq_event_create(void** ev) {
    if (!ev) return DQ_EINVAL;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return DQ_EDEVICE;
    *ev = reinterpret_cast<void*>(e);
    return DQ_OK;
}

dq_status dq_event_destroy(void* ev) {
    if (!ev) return DQ_EINVAL;
    return hipEventDestroy(reinterpret_cast<hipEvent_t>(ev)) == hipSuccess ? DQ_OK : DQ_EDEVICE;
}

dq_status dq_event_elapsed_ms(void* ev_before, void* ev_after, float* ms) {
    if (!ev_before || !ev_after || !ms) return DQ_EINVAL;
    if (hipEventSynchronize(reinterpret_cast<hipEvent_t>(ev_after)) != hipSuccess) return DQ_EDEVICE;
    return hipEventElapsedTime(ms, reinterpret_cast<hipEvent_t>(ev_before),
                               reinterpret_cast<hipEvent_t>(ev_after)) == hipSuccess
               ? DQ_OK
               : DQ_EDEVICE;
}

const char* dq_strerror(int status) {
    switch (status) {
    case DQ_OK: return "ok";
    case DQ_EINVAL: return "invalid argument";
    case DQ_ERANGE: return "value out of range (non-finite input or |q| > 2^31-1)";
    case DQ_ECAPACITY: return "more outliers than the outlier capacity";
    case DQ_ENOTSUP: return "configuration not supported by the GPU kernels";
    case DQ_EDEVICE: return "HIP runtime error";
    case DQ_ECORRUPT: return "codes and outliers are inconsistent";
    case DQ_ENOSCRATCH: return "the call needs more workspace than dq_compress_noalloc's fixed scratch holds";
    default: return "unknown status";
    }
}

}  // extern "C"
