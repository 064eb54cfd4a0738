// dq_kernels.hpp - kernel configurations and launchers of libdq.
#pragma once

#include "dq_device.hpp"

// Every (ndim, B, V) the encode/decode kernels are built for. V is the number
// of consecutive x cells per lane (vector width of the loads); the host picks
// the widest V that divides the row length and matches buffer alignment.
//   1-D: B = 1..4096, V <= B
//   2-D: B = 1..256,  V <= B, B <= 64 V (a block row fits one wave step)
//   3-D: B = 1..64,   V <= B, B <= 64 V, B V <= 64 (plane carry in registers)
#define DQ_CONFIGS(X)                                                            \
    X(1, 1, 1) X(1, 2, 1) X(1, 2, 2) X(1, 4, 1) X(1, 4, 2) X(1, 4, 4)              \
    X(1, 8, 1) X(1, 8, 2) X(1, 8, 4) X(1, 16, 1) X(1, 16, 2) X(1, 16, 4)          \
    X(1, 32, 1) X(1, 32, 2) X(1, 32, 4) X(1, 64, 1) X(1, 64, 2) X(1, 64, 4)       \
    X(1, 128, 1) X(1, 128, 2) X(1, 128, 4) X(1, 256, 1) X(1, 256, 2) X(1, 256, 4) \
    X(1, 512, 1) X(1, 512, 2) X(1, 512, 4) X(1, 1024, 1) X(1, 1024, 2)            \
    X(1, 1024, 4) X(1, 2048, 1) X(1, 2048, 2) X(1, 2048, 4) X(1, 4096, 1)         \
    X(1, 4096, 2) X(1, 4096, 4)                                                  \
    X(2, 1, 1) X(2, 2, 1) X(2, 2, 2) X(2, 4, 1) X(2, 4, 2) X(2, 4, 4)              \
    X(2, 8, 1) X(2, 8, 2) X(2, 8, 4) X(2, 16, 1) X(2, 16, 2) X(2, 16, 4)          \
    X(2, 32, 1) X(2, 32, 2) X(2, 32, 4) X(2, 64, 1) X(2, 64, 2) X(2, 64, 4)       \
    X(2, 128, 2) X(2, 128, 4) X(2, 256, 4)                                       \
    X(3, 1, 1) X(3, 2, 1) X(3, 2, 2) X(3, 4, 1) X(3, 4, 2) X(3, 4, 4)              \
    X(3, 8, 1) X(3, 8, 2) X(3, 8, 4) X(3, 16, 1) X(3, 16, 2) X(3, 16, 4)          \
    X(3, 32, 1) X(3, 32, 2) X(3, 64, 1)

namespace dq {

// The encode and decode sources are compiled once per dimensionality (macro
// DQ_DIM = 1, 2, 3) so the instantiations build in parallel; each object
// defines the launchers of its own dimensionality. They return false when
// (block, v) is not a built configuration.
bool launch_encode_dim1(int block, int v, const EncArgs& a, dim3 grid, hipStream_t stream);
bool launch_encode_dim2(int block, int v, const EncArgs& a, dim3 grid, hipStream_t stream);
bool launch_encode_dim3(int block, int v, const EncArgs& a, dim3 grid, hipStream_t stream);
bool launch_decode_dim1(int block, int v, const DecArgs& a, dim3 grid, hipStream_t stream, bool nt_codes);
bool launch_decode_dim2(int block, int v, const DecArgs& a, dim3 grid, hipStream_t stream, bool nt_codes);
bool launch_decode_dim3(int block, int v, const DecArgs& a, dim3 grid, hipStream_t stream, bool nt_codes);

// Workgroups of the encode kernel that fit on one compute unit at once (0 if
// not built or unknown); one workgroup holds one wave per SIMD.
int encode_occupancy_dim1(int block, int v);
int encode_occupancy_dim2(int block, int v);
int encode_occupancy_dim3(int block, int v);
inline int encode_occupancy(int dim, int block, int v) {
    return dim == 1 ? encode_occupancy_dim1(block, v)
         : dim == 2 ? encode_occupancy_dim2(block, v)
         : dim == 3 ? encode_occupancy_dim3(block, v) : 0;
}

inline bool launch_encode(int dim, int block, int v, const EncArgs& a, dim3 grid, hipStream_t stream) {
    return dim == 1 ? launch_encode_dim1(block, v, a, grid, stream)
         : dim == 2 ? launch_encode_dim2(block, v, a, grid, stream)
         : dim == 3 ? launch_encode_dim3(block, v, a, grid, stream) : false;
}
// nt_codes: nontemporal code loads (every row of the codes starts on a 128-byte line)
inline bool launch_decode(int dim, int block, int v, const DecArgs& a, dim3 grid, hipStream_t stream, bool nt_codes) {
    return dim == 1 ? launch_decode_dim1(block, v, a, grid, stream, nt_codes)
         : dim == 2 ? launch_decode_dim2(block, v, a, grid, stream, nt_codes)
         : dim == 3 ? launch_decode_dim3(block, v, a, grid, stream, nt_codes) : false;
}

// Blocks per tile along x of a configuration (0 if not built).
#define DQ_BPT_CASE(D, BB, VV) \
    if (dim == D && block == BB && v == VV) return Cfg<D, BB, VV>::BPT;
inline int tile_blocks(int dim, int block, int v) {
    DQ_CONFIGS(DQ_BPT_CASE)
    return 0;
}
#undef DQ_BPT_CASE

#define DQ_CAT_(a, b) a##b
#define DQ_CAT(a, b) DQ_CAT_(a, b)

struct AuxArgs {
    const float* x;
    Scalars* sc;
    int32_t* status;
    uint64_t N;
};

constexpr int kMinmaxParts = kBoundParts;  // value-range partials (one per workgroup)
constexpr int kMinmaxThreads = 1024;

void launch_compress_init(Scalars* sc, void* res, double eb, hipStream_t stream);
int launch_minmax(const AuxArgs& a, uint2* parts, void* res, hipStream_t stream);
void launch_sumq(const AuxArgs& a, const BoundArgs& bound, hipStream_t stream);
constexpr uint32_t kChunkTiles = 256;  // tiles per chunk of the large-field scan
constexpr uint32_t kChunkSplit = 8;    // workgroups sharing a chunk's scatter
void launch_chunked_place(const Staging& stg, const Scalars* sc, void* res, uint64_t out_cap,
                          const uint32_t* tile_count, uint32_t* tile_off, uint32_t* chunk_sum, uint32_t n_tiles,
                          const uint32_t* block_info, Geom g, uint32_t* out_idx, int32_t* out_val,
                          hipStream_t stream);
constexpr uint32_t kPlaceTiles = 8192;  // tiles the fused scan + scatter holds in LDS
void launch_place(const Staging& stg, const Scalars* sc, void* res, uint64_t out_cap, const uint32_t* tile_count,
                  uint32_t n_tiles, const uint32_t* block_info, Geom g, uint32_t* out_idx, int32_t* out_val,
                  hipStream_t stream);
void launch_index(const uint32_t* out_idx, uint32_t n_out, Geom g, int block_log2, int dim,
                  uint32_t* block_start, void* res, uint32_t tag, hipStream_t stream, const void* src = nullptr,
                  uint32_t cap = 0);
void launch_result_reset(void* res, hipStream_t stream);

// ---------------------------------------------------------------- batches

// Per-field arguments of the batched value-range pass / bound record.
struct AuxField {
    const float* x;
    uint64_t N;
    uint2* parts;
    Scalars* sc;
    void* res_;       // the compress dq_result (device)
    double eb;        // absolute bound (nparts == 0)
    int nparts;       // 0: absolute bound, no value-range pass: initialisation only
    int vec4;
    unsigned long long* dres_word;  // the decompress result's status word
};

// Per-field arguments of the batched placement (dense staging).
struct PlaceField {
    Staging stg;
    void* res_;
    uint64_t out_cap;
    const uint32_t* cnt;  // tile outlier counts
    uint32_t* tile_off;
    uint32_t* chunk_sum;
    uint32_t n_tiles, n_chunks;
    const uint32_t* block_info;
    Geom g;
    uint32_t* out_idx;
    int32_t* out_val;
};

// Value-range passes of every field, then each field's range reduced to the
// pair reduced[2 * field] (16-byte aligned slots, 2 uint2 per field).
void launch_batch_aux(const AuxField* fields, uint32_t n_fields, const uint2* units, uint32_t n_units,
                      unsigned int* tickets, uint32_t n_tickets, uint2* reduced, hipStream_t stream);
void launch_batch_place(const PlaceField* fields, const uint2* units, uint32_t n_units, hipStream_t stream);

// Persistent batch encode / decode of one (dim, block, v) class; grid =
// min(units, resident workgroups). False if the class is not built.
bool launch_encode_batch_dim1(int block, int v, const BatchQueue& q, int grid, hipStream_t stream);
bool launch_encode_batch_dim2(int block, int v, const BatchQueue& q, int grid, hipStream_t stream);
bool launch_encode_batch_dim3(int block, int v, const BatchQueue& q, int grid, hipStream_t stream);
bool launch_decode_batch_dim1(int block, int v, const BatchQueue& q, int grid, hipStream_t stream);
bool launch_decode_batch_dim2(int block, int v, const BatchQueue& q, int grid, hipStream_t stream);
bool launch_decode_batch_dim3(int block, int v, const BatchQueue& q, int grid, hipStream_t stream);
inline bool launch_encode_batch(int dim, int block, int v, const BatchQueue& q, int grid, hipStream_t stream) {
    return dim == 1 ? launch_encode_batch_dim1(block, v, q, grid, stream)
         : dim == 2 ? launch_encode_batch_dim2(block, v, q, grid, stream)
         : dim == 3 ? launch_encode_batch_dim3(block, v, q, grid, stream) : false;
}
inline bool launch_decode_batch(int dim, int block, int v, const BatchQueue& q, int grid, hipStream_t stream) {
    return dim == 1 ? launch_decode_batch_dim1(block, v, q, grid, stream)
         : dim == 2 ? launch_decode_batch_dim2(block, v, q, grid, stream)
         : dim == 3 ? launch_decode_batch_dim3(block, v, q, grid, stream) : false;
}

}  // namespace dq
