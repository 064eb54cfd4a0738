// dq_batch.hip - a batch of fields as one HIP graph (host runtime, no kernels
// of its own): the fields' compress and device-count decompress calls are
// captured once over parallel branches and replayed with one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <array>
#include <numeric>
#include <vector>

#include "../../include/dq.h"
#include "../../include/dq_batch.h"
#include "dq_host.hpp"

struct dq_batch_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> streams;  // [0] capture origin, then the branches
    std::vector<hipEvent_t> events;    // [0] fork, then one join per branch
    // persistent batches: the launch sequence, enqueued on one stream
    // (timing hooks around the largest class's kernels) or with branches
    std::function<dq_status(hipStream_t, bool, const dq_hooks*, const dq_hooks*)> enqueue;
};

namespace {

void release(dq_batch_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    for (hipStream_t s : g->streams) (void)hipStreamDestroy(s);
    delete g;
}

uint64_t cells(const dq_params& p) {
    uint64_t n = 1;
    for (int a = 0; a < p.ndim && a < 3; ++a) n *= (uint64_t)(p.shape[a] > 0 ? p.shape[a] : 0);
    return n;
}

// ------------------------------------------------------------------ persistent batches

using namespace dq;
using namespace dq::host;

constexpr uint32_t kUnitTiles = 4 * kWaves;  // tiles per ticket (workgroup) of the persistent encode / decode

// The queue and field tables of a persistent batch, in the caller's workspace.
struct PersistentLayout {
    uint64_t enc, dec, aux, place, aux_units, chunk_units, class_units, tickets, reduced, total;
    uint32_t n_aux_units, n_chunk_units, n_class_units;
    std::vector<int> cls;                          // class of every field
    std::vector<std::array<int, 3>> classes;       // (dim, block, v)
    std::vector<Plan> plans;
};

int minmax_parts(uint64_t N, bool vec4) {
    const uint64_t work = vec4 ? N / 4 : N;
    uint64_t b = (work + 4 * kMinmaxThreads - 1) / (4 * kMinmaxThreads);
    if (b > (uint64_t)kMinmaxParts) b = kMinmaxParts;
    return (int)(b < 1 ? 1 : b);
}

bool needs_range(const dq_params& p) {
    return p.eb_mode == DQ_EB_REL || p.pad_mode == DQ_PAD_GLOBAL_MIN || p.pad_mode == DQ_PAD_GLOBAL_MAX;
}

// Checks every field and plans the batch (no device access).
dq_status persistent_plan(const dq_batch_field* fields, uint64_t n, PersistentLayout& L) {
    if (!fields || n == 0 || n > 0xffffffffull) return DQ_EINVAL;
    L.plans.resize(n);
    L.cls.resize(n);
    uint64_t aux_units = 0, chunk_units = 0, class_units = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const dq_batch_field& f = fields[i];
        const dq_params* p = &f.p;
        dq_status st = validate(p, true);
        if (st != DQ_OK) return st;
        uint64_t npads = 0;
        dq_pad_count(p, &npads);
        if (!f.x || !f.codes || !f.out_idx || !f.out_val || !f.cres || !f.cws || !f.x_hat || !f.dres)
            return DQ_EINVAL;
        if (npads > 0 && !f.pads) return DQ_EINVAL;
        if ((reinterpret_cast<uintptr_t>(f.cres) % 8) || (reinterpret_cast<uintptr_t>(f.dres) % 8) ||
            (reinterpret_cast<uintptr_t>(f.cws) % kAlign))
            return DQ_EINVAL;
        if (p->pad_mode == DQ_PAD_GLOBAL_MEAN) return DQ_ENOTSUP;  // needs its own pass over q
        Plan pl;
        if (!make_plan(p, f.x, f.codes, pl)) return DQ_ENOTSUP;
        Geom g0;
        base_geom(p, g0);
        if (f.out_cap < g0.N) return DQ_ENOTSUP;  // dense staging only
        const CompressLayout cl = compress_layout(p, f.out_cap);
        if (f.cws_bytes < cl.total) return DQ_EINVAL;
        // the decode runs on the compress call's tiling, so x_hat must allow
        // its V too; and every tile's region must hold a slot per cell of its
        // blocks (dense staging): else fewer cells per lane
        const uint32_t bcells = (uint32_t)pl.B * (pl.dim >= 2 ? (uint32_t)pl.B : 1u) * (pl.dim == 3 ? (uint32_t)pl.B : 1u);
        auto fits = [&](const Plan& q) {
            const uint64_t spt = cl.cap / q.g.n_tiles;
            const uint64_t tile_blocks_max = q.g.bpt < q.g.nbx ? q.g.bpt : q.g.nbx;
            return reinterpret_cast<uintptr_t>(f.x_hat) % (4u * (uint32_t)q.V) == 0 && spt > 0 &&
                   tile_blocks_max * bcells <= 2ull * spt;
        };
        while (!fits(pl)) {
            if (pl.V == 1 || !finish_plan(p, pl.V / 2, pl)) return DQ_ENOTSUP;
        }
        L.plans[i] = pl;
        const std::array<int, 3> key{pl.dim, pl.B, pl.V};
        int c = -1;
        for (size_t k = 0; k < L.classes.size(); ++k)
            if (L.classes[k] == key) c = (int)k;
        if (c < 0) {
            c = (int)L.classes.size();
            L.classes.push_back(key);
        }
        L.cls[i] = c;
        const bool vec4 = (reinterpret_cast<uintptr_t>(f.x) & 15u) == 0;
        aux_units += needs_range(*p) ? (uint64_t)minmax_parts(pl.g.N, vec4) : 1u;
        chunk_units += (pl.g.n_tiles + kChunkTiles - 1) / kChunkTiles;
        class_units += (pl.g.n_tiles + kUnitTiles - 1) / kUnitTiles;
    }
    if (aux_units > 0xffffffffull || chunk_units * kChunkSplit > 0xffffffffull || class_units > 0xffffffffull)
        return DQ_ENOTSUP;
    L.n_aux_units = (uint32_t)aux_units;
    L.n_chunk_units = (uint32_t)chunk_units;
    L.n_class_units = (uint32_t)class_units;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off += align_up(bytes);
        return o;
    };
    L.enc = take(sizeof(EncArgs) * n);
    L.dec = take(sizeof(DecArgs) * n);
    L.aux = take(sizeof(AuxField) * n);
    L.place = take(sizeof(PlaceField) * n);
    L.aux_units = take(sizeof(uint2) * aux_units);
    L.chunk_units = take(sizeof(uint2) * chunk_units);
    L.class_units = take(2 * sizeof(uint4) * class_units);  // encode units, then decode units, class by class
    L.tickets = take(sizeof(unsigned int) * 2 * L.classes.size());
    L.reduced = take(sizeof(uint4) * n);  // one 16-byte (min key, max key) slot per field
    L.total = off;
    return DQ_OK;
}

}  // namespace

extern "C" {

dq_status dq_batch_persistent_workspace(const dq_batch_field* fields, uint64_t n, uint64_t* bytes) {
    if (!bytes) return DQ_EINVAL;
    PersistentLayout L;
    const dq_status st = persistent_plan(fields, n, L);
    if (st != DQ_OK) return st;
    *bytes = L.total;
    return DQ_OK;
}

dq_status dq_batch_persistent_create(const dq_batch_field* fields, uint64_t n, void* ws, uint64_t ws_bytes,
                                     int32_t* class_out, int32_t* vec_out, dq_batch_graph** graph) {
    if (!graph) return DQ_EINVAL;
    *graph = nullptr;
    PersistentLayout L;
    dq_status st = persistent_plan(fields, n, L);
    if (st != DQ_OK) return st;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) || ws_bytes < L.total) return DQ_EINVAL;
    char* w = static_cast<char*>(ws);
    // the tables, built on the host
    std::vector<EncArgs> enc(n);
    std::vector<DecArgs> dec(n);
    std::vector<AuxField> aux(n);
    std::vector<PlaceField> place(n);
    std::vector<uint2> aux_units, chunk_units;
    std::vector<std::vector<uint4>> cunits(L.classes.size());
    for (uint64_t i = 0; i < n; ++i) {
        const dq_batch_field& f = fields[i];
        const dq_params* p = &f.p;
        const Plan& pl = L.plans[i];
        const CompressLayout cl = compress_layout(p, f.out_cap);
        char* cw = static_cast<char*>(f.cws);
        Scalars* sc = reinterpret_cast<Scalars*>(cw + cl.sc);
        uint32_t* tiles = reinterpret_cast<uint32_t*>(cw + cl.tiles);
        uint32_t* toff = reinterpret_cast<uint32_t*>(cw + cl.toff);
        uint32_t* csum = reinterpret_cast<uint32_t*>(cw + cl.csum);
        uint32_t* info = reinterpret_cast<uint32_t*>(cw + cl.info);
        uint2* parts = reinterpret_cast<uint2*>(cw + cl.parts);
        Staging stg;
        stg.spt = (uint32_t)(cl.cap / pl.g.n_tiles);
        stg.region = reinterpret_cast<uint4*>(cw + cl.region);
        stg.ovf = reinterpret_cast<uint4*>(cw + cl.ovf);
        stg.ovf_cap = (uint32_t)cl.cap;
        stg.bcells = (uint32_t)pl.B * (pl.dim >= 2 ? (uint32_t)pl.B : 1u) * (pl.dim == 3 ? (uint32_t)pl.B : 1u);
        stg.dense = 1u;
        const bool vec4 = (reinterpret_cast<uintptr_t>(f.x) & 15u) == 0;
        const int nparts = needs_range(*p) ? minmax_parts(pl.g.N, vec4) : 0;
        EncArgs& ea = enc[i];
        // the encode reads the field's range as one pair, reduced after the value-range pass
        const uint2* range = nparts ? reinterpret_cast<const uint2*>(w + L.reduced) + 2 * i : parts;
        ea.bound = BoundArgs{range, nparts ? 1 : 0, p->eb, p->eb_mode == DQ_EB_REL ? 1 : 0};
        ea.eb_out = &f.cres->eb_abs;
        ea.x = f.x;
        ea.codes = f.codes;
        ea.pads = f.pads;
        ea.block_info = info;
        ea.tile_count = tiles;
        ea.stg = stg;
        ea.sc = sc;
        ea.status = &f.cres->status;
        ea.g = pl.g;
        ea.R = p->radius;
        ea.pad_mode = p->pad_mode;
        DecArgs& da = dec[i];
        da.src = reinterpret_cast<const ResultView*>(f.cres);
        da.cap = (uint32_t)cl.cap;
        da.res_word = reinterpret_cast<unsigned long long*>(f.dres);
        da.n_out_out = reinterpret_cast<unsigned long long*>(&f.dres->n_out);
        da.eb_out = &f.dres->eb_abs;
        da.eb_abs = 1.0;
        da.tag = next_tag();
        da.codes = f.codes;
        da.out_idx = f.out_idx;
        da.out_val = f.out_val;
        da.pads = f.pads;
        da.block_start = nullptr;
        da.tile_off = toff;
        da.tile_count = tiles;
        da.block_info = info;
        da.x_hat = f.x_hat;
        da.g = pl.g;
        da.twoeb = 2.0;
        da.n_out = 0;
        da.R = p->radius;
        da.pad_mode = p->pad_mode;
        AuxField& af = aux[i];
        af.x = f.x;
        af.N = pl.g.N;
        af.parts = parts;
        af.sc = sc;
        af.res_ = f.cres;
        af.eb = p->eb;
        af.nparts = nparts;
        af.vec4 = vec4 ? 1 : 0;
        af.dres_word = reinterpret_cast<unsigned long long*>(f.dres);
        for (int k = 0; k < (af.nparts ? af.nparts : 1); ++k) aux_units.push_back(make_uint2((uint32_t)i, (uint32_t)k));
        PlaceField& pf = place[i];
        pf.stg = stg;
        pf.res_ = f.cres;
        pf.out_cap = f.out_cap;
        pf.cnt = tiles;
        pf.tile_off = toff;
        pf.chunk_sum = csum;
        pf.n_tiles = pl.g.n_tiles;
        pf.n_chunks = (pl.g.n_tiles + kChunkTiles - 1) / kChunkTiles;
        pf.block_info = info;
        pf.g = pl.g;
        pf.out_idx = f.out_idx;
        pf.out_val = f.out_val;
        for (uint32_t c = 0; c < pf.n_chunks; ++c) chunk_units.push_back(make_uint2((uint32_t)i, c));
        for (uint32_t t = 0; t < pl.g.n_tiles; t += kUnitTiles)
            cunits[L.cls[i]].push_back(make_uint4((uint32_t)i, t, std::min(kUnitTiles, pl.g.n_tiles - t), 0u));
    }
    // class units: encode units of every class, then the same again for decode
    std::vector<uint4> all_units;
    std::vector<uint64_t> class_first;
    for (const auto& v : cunits) {
        class_first.push_back(all_units.size());
        all_units.insert(all_units.end(), v.begin(), v.end());
    }
    const uint64_t n_units = all_units.size();
    all_units.insert(all_units.end(), all_units.begin(), all_units.begin() + (ptrdiff_t)n_units);
    auto put = [&](uint64_t off, const void* src, uint64_t bytes) {
        return bytes == 0 || hipMemcpy(w + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!put(L.enc, enc.data(), sizeof(EncArgs) * n) || !put(L.dec, dec.data(), sizeof(DecArgs) * n) ||
        !put(L.aux, aux.data(), sizeof(AuxField) * n) || !put(L.place, place.data(), sizeof(PlaceField) * n) ||
        !put(L.aux_units, aux_units.data(), sizeof(uint2) * aux_units.size()) ||
        !put(L.chunk_units, chunk_units.data(), sizeof(uint2) * chunk_units.size()) ||
        !put(L.class_units, all_units.data(), sizeof(uint4) * all_units.size()))
        return DQ_EDEVICE;

    // the classes' encode (and decode) kernels are independent: one graph
    // branch per class, so one class's tail overlaps another's work
    const uint32_t ncls = (uint32_t)L.classes.size();
    dq_batch_graph* g = new dq_batch_graph();
    for (uint32_t k = 0; k <= ncls; ++k) {
        hipStream_t bs;
        if (hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) != hipSuccess) {
            release(g);
            return DQ_EDEVICE;
        }
        g->streams.push_back(bs);
    }
    for (uint32_t k = 0; k < 2 * (ncls + 1); ++k) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            release(g);
            return DQ_EDEVICE;
        }
        g->events.push_back(e);
    }
    // the class with the most cells carries the timing hooks
    std::vector<uint64_t> class_cells(ncls, 0);
    for (uint64_t i = 0; i < n; ++i) class_cells[L.cls[i]] += L.plans[i].g.N;
    const uint32_t big = (uint32_t)(std::max_element(class_cells.begin(), class_cells.end()) - class_cells.begin());
    for (uint64_t i = 0; i < n; ++i) {  // the hooked class is reported as class 0
        const uint32_t c = (uint32_t)L.cls[i];
        if (class_out) class_out[i] = c == big ? 0 : (int32_t)(c < big ? c + 1 : c);
        if (vec_out) vec_out[i] = L.plans[i].V;
    }
    std::vector<uint32_t> class_units(ncls);
    for (uint32_t c = 0; c < ncls; ++c) class_units[c] = (uint32_t)cunits[c].size();
    const std::vector<std::array<int, 3>> classes = L.classes;
    const PersistentLayout lay = L;
    // The launch sequence. branch = true: the classes' encode (and decode)
    // kernels on parallel streams forked from s and joined back (the graph);
    // false: everything on s in order, the hooks around the largest class.
    const uint32_t n_fields = (uint32_t)n;
    g->enqueue = [g, w, lay, classes, class_first, class_units, n_units, ncls, big, n_fields](
                     hipStream_t s, bool branch, const dq_hooks* enc_hooks, const dq_hooks* dec_hooks) -> dq_status {
        dq_status rst = DQ_OK;
        unsigned int* tickets = reinterpret_cast<unsigned int*>(w + lay.tickets);
        const uint4* units = reinterpret_cast<const uint4*>(w + lay.class_units);
        auto queue = [&](uint32_t c, bool decode) {
            BatchQueue q;
            q.enc = reinterpret_cast<const EncArgs*>(w + lay.enc);
            q.dec = reinterpret_cast<const DecArgs*>(w + lay.dec);
            q.units = units + (decode ? n_units : 0) + class_first[c];
            q.n_units = class_units[c];
            q.ticket = tickets + 2 * c + (decode ? 1 : 0);
            return q;
        };
        auto hook = [&](const dq_hooks* h, bool after, hipStream_t bs) {
            void* e = h ? (after ? h->ev_after : h->ev_before) : nullptr;
            if (e) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(e), bs);
        };
        // fork the class branches off s (events [phase * (ncls + 1)]), run f
        // on branch c, join them back (events [phase * (ncls + 1) + 1 + c])
        auto phase = [&](int ph, auto&& f) {
            if (!branch) {
                for (uint32_t c = 0; c < ncls; ++c)
                    if (!f(c, s)) rst = DQ_ENOTSUP;
                return;
            }
            hipEvent_t fork = g->events[ph * (ncls + 1)];
            bool ok = hipEventRecord(fork, s) == hipSuccess;
            for (uint32_t c = 0; ok && c < ncls; ++c) {
                hipStream_t bs = g->streams[1 + c];
                ok = hipStreamWaitEvent(bs, fork, 0) == hipSuccess;
                if (ok && !f(c, bs)) rst = DQ_ENOTSUP;
                hipEvent_t join = g->events[ph * (ncls + 1) + 1 + c];
                ok = ok && hipEventRecord(join, bs) == hipSuccess && hipStreamWaitEvent(s, join, 0) == hipSuccess;
            }
            if (!ok && rst == DQ_OK) rst = DQ_EDEVICE;
        };
        launch_batch_aux(reinterpret_cast<const AuxField*>(w + lay.aux), n_fields,
                         reinterpret_cast<const uint2*>(w + lay.aux_units), lay.n_aux_units, tickets, 2 * ncls,
                         reinterpret_cast<uint2*>(w + lay.reduced), s);
        phase(0, [&](uint32_t c, hipStream_t bs) {
            const BatchQueue q = queue(c, false);
            if (c == big) hook(enc_hooks, false, bs);
            const bool ok = launch_encode_batch(classes[c][0], classes[c][1], classes[c][2], q, (int)q.n_units, bs);
            if (c == big) hook(enc_hooks, true, bs);
            return ok;
        });
        launch_batch_place(reinterpret_cast<const PlaceField*>(w + lay.place),
                           reinterpret_cast<const uint2*>(w + lay.chunk_units), lay.n_chunk_units, s);
        phase(1, [&](uint32_t c, hipStream_t bs) {
            const BatchQueue q = queue(c, true);
            if (c == big) hook(dec_hooks, false, bs);
            const bool ok = launch_decode_batch(classes[c][0], classes[c][1], classes[c][2], q, (int)q.n_units, bs);
            if (c == big) hook(dec_hooks, true, bs);
            return ok;
        });
        if (rst == DQ_OK && hipGetLastError() != hipSuccess) rst = DQ_EDEVICE;
        return rst;
    };
    hipStream_t s = g->streams[0];
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
        release(g);
        return DQ_EDEVICE;
    }
    st = g->enqueue(s, true, nullptr, nullptr);
    hipGraph_t captured = nullptr;
    const bool ended = hipStreamEndCapture(s, &captured) == hipSuccess;
    g->graph = captured;
    if (st == DQ_OK && !ended) st = DQ_EDEVICE;
    if (st == DQ_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) st = DQ_EDEVICE;
    if (st != DQ_OK) {
        (void)hipGetLastError();
        release(g);
        return st;
    }
    *graph = g;
    return DQ_OK;
}

}  // extern "C"

extern "C" {

dq_status dq_batch_graph_create(const dq_batch_field* fields, uint64_t n, int branches, dq_batch_graph** graph) {
    if (!fields || n == 0 || !graph || branches < 1 || branches > 16) return DQ_EINVAL;
    *graph = nullptr;
    for (uint64_t i = 0; i < n; ++i) {
        const dq_status st = dq_validate(&fields[i].p);
        if (st != DQ_OK) return st;
    }
    dq_batch_graph* g = new dq_batch_graph();
    const int nb = (int)std::min<uint64_t>((uint64_t)branches, n);
    for (int k = 0; k <= nb; ++k) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            release(g);
            return DQ_EDEVICE;
        }
        g->streams.push_back(s);
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            release(g);
            return DQ_EDEVICE;
        }
        g->events.push_back(e);
    }
    // largest fields first, each to the least loaded branch
    std::vector<uint64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint64_t a, uint64_t b) { return cells(fields[a].p) > cells(fields[b].p); });
    std::vector<uint64_t> load(nb, 0);
    std::vector<int> branch_of(n, 0);
    for (uint64_t i : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        branch_of[i] = b;
        load[b] += cells(fields[i].p);
    }

    hipStream_t origin = g->streams[0];
    if (hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed) != hipSuccess) {
        release(g);
        return DQ_EDEVICE;
    }
    dq_status st = DQ_OK;
    bool ok = hipEventRecord(g->events[0], origin) == hipSuccess;
    for (int b = 0; ok && b < nb; ++b) ok = hipStreamWaitEvent(g->streams[1 + b], g->events[0], 0) == hipSuccess;
    if (!ok) st = DQ_EDEVICE;
    for (uint64_t i : order) {
        if (st != DQ_OK) break;
        const dq_batch_field& f = fields[i];
        void* s = g->streams[1 + branch_of[i]];
        st = dq_compress(&f.p, f.x, f.codes, f.out_idx, f.out_val, f.out_cap, f.pads, f.cres, f.cws, f.cws_bytes, s,
                         nullptr);
        if (st == DQ_OK && f.x_hat)
            st = dq_decompress_dev(&f.p, f.cres, f.out_cap, f.codes, f.out_idx, f.out_val, f.pads, f.x_hat, f.dres,
                                   f.dws, f.dws_bytes, s, nullptr);
    }
    for (int b = 0; st == DQ_OK && b < nb; ++b) {
        if (hipEventRecord(g->events[1 + b], g->streams[1 + b]) != hipSuccess ||
            hipStreamWaitEvent(origin, g->events[1 + b], 0) != hipSuccess)
            st = DQ_EDEVICE;
    }
    hipGraph_t captured = nullptr;
    const bool ended = hipStreamEndCapture(origin, &captured) == hipSuccess;
    g->graph = captured;
    if (st == DQ_OK && !ended) st = DQ_EDEVICE;
    if (st == DQ_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) st = DQ_EDEVICE;
    if (st != DQ_OK) {
        (void)hipGetLastError();
        release(g);
        return st;
    }
    *graph = g;
    return DQ_OK;
}

dq_status dq_batch_graph_launch(dq_batch_graph* graph, void* hip_stream) {
    if (!graph || !graph->exec) return DQ_EINVAL;
    return hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(hip_stream)) == hipSuccess ? DQ_OK
                                                                                                  : DQ_EDEVICE;
}

dq_status dq_batch_persistent_run(dq_batch_graph* graph, void* hip_stream, const dq_hooks* enc_hooks,
                                  const dq_hooks* dec_hooks) {
    if (!graph || !graph->enqueue) return DQ_EINVAL;
    return graph->enqueue(reinterpret_cast<hipStream_t>(hip_stream), false, enc_hooks, dec_hooks);
}

dq_status dq_batch_graph_destroy(dq_batch_graph* graph) {
    if (!graph) return DQ_EINVAL;
    release(graph);
    return DQ_OK;
}

}  // extern "C"
