// dq_host.hpp - host-side planning shared by libdq's entry points: parameter
// checks, the tiling of a field, the compress workspace layout, call tags.
#pragma once

#include "../../include/dq.h"
#include "dq_kernels.hpp"

namespace dq {
namespace host {

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// The tiling of one call: geometry, dimensionality, block edge, cells per lane.
struct Plan {
    Geom g;
    int dim, B, V;
    uint64_t nblocks;
};

// Compress workspace: scalars, value-range partials, per-tile counts and
// offsets, per-chunk count sums, per-block outlier prefixes, then the outlier
// staging area: per-tile regions of cap entries in all (cap / tiles each),
// and an overflow list of cap entries (the overflow never exceeds the outlier
// count, so everything fits whenever the outliers fit the caller's capacity).
struct CompressLayout {
    uint64_t sc, parts, tiles, toff, csum, info, region, ovf, cap, total;
};

int ilog2(uint32_t v);
// Host check shared by every entry point; check_eb is false for decompress.
dq_status validate(const dq_params* p, bool check_eb);
void base_geom(const dq_params* p, Geom& g);
// The tiling with V cells per lane (false if not built or not possible).
bool finish_plan(const dq_params* p, int V, Plan& pl);
// The hinted or automatic V for a field buffer fptr and code buffer cptr.
bool make_plan(const dq_params* p, const void* fptr, const void* cptr, Plan& pl);
CompressLayout compress_layout(const dq_params* p, uint64_t out_cap);
// A tag distinct for every call of the process, never 0.
uint32_t next_tag();
// True when every row of the codes starts on a 128-byte line (an aligned
// buffer, and rows of a multiple of 64 cells in 2-D and 3-D): the decode then
// loads the codes nontemporally (see the note on codes in dq_device.hpp).
bool codes_rows_on_lines(const Geom& g, int dim, const void* codes);

}  // namespace host
}  // namespace dq
