// Internal structures shared by the C-ABI layer (api.cpp, table.cpp) and
// the HIP kernels (step.hip, surrogate.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "qedmi.h"
#include "surrogate.hpp"

namespace qedmi {

constexpr int kMaxSets = 8;
constexpr int kBlock = 256;               // threads per block of the step kernels
constexpr int kChunk = 4096;              // particles per chunk (16 per thread)
constexpr int kMasks = kChunk / 64;       // 64-bit event masks per chunk
constexpr int kMaxTableChi = 1024;        // 1D table points staged in LDS
constexpr int kStatusBits = 30;           // value bits of a look-back status word

void set_error(const std::string& msg);

// Device view of one lookup table ("table view": non-owning pointers passed
// by value to kernels).
// The CDF arrays are in row-pair order: entry (n, k), n < n_chi - 1, holds
// (P[n][k], P[n+1][k]) at [2 (n n_frac + k)] and [2 (n n_frac + k) + 1].
struct TableDev {
    const double* ln_rate64;
    const double* cdf64;
    const float* ln_rate32;
    const float* cdf32;
    const uint16_t* ln_rate16;
    const uint16_t* cdf16;
    int32_t n_chi, n_frac;
    double chi_min, chi_max;
    double ln_chi_min, inv_dlnchi;   // t = (ln chi - ln chi_min) * inv_dlnchi
    double frac_min, ln_frac_min;
    double inv_chi_min, ln_chi_max;
    // The same parameters rounded to FP32 on the host: FP32 kernels read
    // them as uniform kernel arguments (scalar registers) instead of
    // converting the FP64 ones into vector registers that live across the
    // particle loops.
    float chi_min_f, chi_max_f, ln_chi_min_f, inv_dlnchi_f, ln_frac_min_f, inv_chi_min_f, ln_chi_max_f;
};

struct SetDev {
    void* p[11];          // ux uy uz ex ey ez bx by bz tau w
    int64_t n, id_base;
    int32_t species;
    int32_t stream;       // 0: emits photons (leptons), 1: makes pairs (photons), -1: ions
    uint8_t* flags;
};

struct AppendDev {
    void *ux, *uy, *uz, *w, *tau;
    int64_t* parent;
    int64_t* count;
    int64_t capacity;
};

// One chunk of <= kChunk consecutive particles of one set.  Chunks are
// ordered by (stream, tile order); each stream's chunks are contiguous.
struct ChunkDesc {
    int64_t begin;
    int32_t set;
    int32_t len;
    int32_t stream;
    int32_t stream_first;   // index of the first chunk of this stream
    int32_t stream_last;    // index of the last chunk of this stream
    int32_t pad_;
};

// Caller units -> the library's (E in V/m, B in T, u = p/(m_e c), t in s,
// energies in m_e c^2).  All 1 for SI.
struct Units {
    double e = 1.0, b = 1.0, u = 1.0, inv_u = 1.0;   // multiply a caller value by these
    float e_f = 1.0f, b_f = 1.0f, u_f = 1.0f, inv_u_f = 1.0f;   // the same, rounded to FP32
    double t = 1.0;        // seconds per caller time unit
    double energy = 1.0;   // m_e c^2 per caller energy unit
    double length = 1.0;   // metres per caller length unit
};

struct StepArgs {
    SetDev sets[kMaxSets];
    int32_t n_sets;
    int32_t n_chunks;
    const ChunkDesc* chunks;
    unsigned long long* status;   // look-back status words, one per chunk
    unsigned long long* ticket;   // monotonically increasing chunk ticket
    unsigned long long ticket_base;
    uint32_t epoch;               // launch tag carried by status words
    int32_t generate_only;        // 1: events from flags, no evolution
    TableDev bw, qs;
    AppendDev ph, el, po;
    int64_t* stats;
    SurrogateDev bw_surr, qs_surr;  // valid when use_*_surr
    int32_t use_bw_surr, use_qs_surr;
    double dt;
    float dt_f;                     // dt rounded to FP32
    unsigned long long seed, step;
    double photon_min_energy;
    int32_t chi_mode;
    double chi_qed_min;             // 0: no classical regime
    double drag;                    // (2/3) (alpha m c^2 / hbar) dt
    Units units;
};

struct ElemArgs {
    SetDev set;
    TableDev table;
    void* chi_out;
    double dt;
    unsigned long long seed;
    int32_t chi_mode;
    int32_t is_photon;
    Units units;
};

// Chunk table construction on the device (chunks.hip).  The host has
// validated the tiles and counted the chunks; `order` / `ostart` are device
// scratch of n_part entries each.
struct ChunkBuildArgs {
    const int64_t* tiles;        // device, 3 * n_tiles; NULL: one tile per set
    int32_t n_tiles;             // tiles (sets when `tiles` is NULL)
    int32_t n_part0;             // tiles of stream 0 holding at least one chunk
    int32_t n_part;              // ... of both streams
    int32_t n_chunks0;           // chunks of stream 0 (they come first)
    int32_t n_chunks;
    int32_t set_stream[kMaxSets];
    int64_t set_n[kMaxSets];
    int32_t* order;              // tile index by position in its stream
    int32_t* ostart;             // first chunk of that tile
    ChunkDesc* chunks;           // n_chunks entries
};
hipError_t launch_chunk_build(const ChunkBuildArgs& a, hipStream_t s);
// Copy host tiles to device memory through kernel arguments (no staging
// buffer, no allocation): one small launch per 160 tiles.
hipError_t store_tiles_by_args(const int64_t* host_tiles, int n_tiles, int64_t* dst, hipStream_t s);

// Kernel launchers (step.hip).  Return hipError_t of the launch.
hipError_t launch_step(const StepArgs& a, int dtype, int grid, hipStream_t s);
hipError_t launch_chi(const ElemArgs& a, int dtype, hipStream_t s);
hipError_t launch_init_tau(const ElemArgs& a, int dtype, hipStream_t s);
hipError_t launch_evolve(const ElemArgs& a, int dtype, hipStream_t s);
int step_grid_size(const StepArgs& a, int dtype, int device);
size_t step_lds_bytes_for(const StepArgs& a, int dtype);

struct TableCallArgs {
    TableDev table;
    const void* a;        // chi
    const void* b;        // gamma (rate) or u (sample)
    void* out;
    uint8_t* sel;
    int64_t n;
    int32_t process;
};
hipError_t launch_table_rate(const TableCallArgs& a, int dtype, hipStream_t s);
hipError_t launch_table_sample(const TableCallArgs& a, int dtype, hipStream_t s);

}  // namespace qedmi

struct qed_table {
    qed_table_params p{};
    std::vector<double> ln_rate, cdf;
    int device = -1;
    double* d_ln_rate64 = nullptr;
    double* d_cdf64 = nullptr;
    float* d_ln_rate32 = nullptr;
    float* d_cdf32 = nullptr;
    uint16_t* d_ln_rate16 = nullptr;
    uint16_t* d_cdf16 = nullptr;
    qedmi::TableDev view() const;
};

struct qed_context {
    int device = -1;
    int cu_count = 0;
    unsigned long long* d_ticket = nullptr;
    unsigned long long* d_status = nullptr;
    int64_t status_cap = 0;
    unsigned long long ticket_issued = 0;   // host mirror of the ticket counter
    uint32_t epoch = 0;
    qedmi::ChunkDesc* d_chunks = nullptr;
    int64_t chunks_cap = 0;
    // device tile list and chunk-builder scratch (order, ostart)
    int64_t* d_tiles = nullptr;
    int32_t* d_part = nullptr;
    int64_t tiles_cap = 0;
    // pinned host staging of the tile list, double-buffered: buffer i is
    // rewritten only after the copy issued from it two calls earlier is done
    int64_t* h_stage[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int64_t stage_cap = 0;
    int stage_next = 0;
    // layout of the chunk table now on the device (skip the rebuild when unchanged)
    bool layout_valid = false;
    std::vector<int64_t> layout_key;
    std::vector<int32_t> tile_idx;          // host scratch of the tile overlap check
    // persistent grid per step-kernel variant (dtype, surrogate, chi mode, LDS bytes)
    struct GridCache {
        int dtype, surr, chi_mode;
        size_t lds;
        int grid;
    };
    std::vector<GridCache> grids;
    void* d_scratch = nullptr;              // general device scratch (Schwinger scan offsets)
    int64_t scratch_cap = 0;                // bytes
    qedmi::Units units;                     // caller unit system (qed_context_set_units)
};

namespace qedmi {
// Shared by the C-ABI translation units (defined in api.cpp).
int32_t check_append_dtype(const qed_append* a, int dtype, const char* name);
AppendDev append_view(const qed_append* a);
int32_t reserve_scratch(qed_context* ctx, int64_t bytes);
// Table generation on the current device (tablegen_device.hip); fills host arrays.
int32_t generate_tables_device(const qed_table_params& p, double* ln_rate, double* cdf, hipStream_t stream);

// Fused-step preparation shared by qed_step and its allocation-free variant.
struct ChunkPlan {
    int32_t n_tiles;        // tiles (sets when the caller gave none)
    int32_t n_part0, n_part;
    int32_t n_chunks0, n_chunks;
};
// Validate a step descriptor and fill the kernel arguments, in two parts:
// the particle sets (no HIP call), then tables, append buffers and
// surrogates.  The chunk table, look-back scratch and ticket are left for
// the caller.  No allocation.
int32_t prepare_sets(const qed_step_desc* d, bool generate_only, StepArgs& a, int& dtype);
int32_t prepare_tables(const Units& units, const qed_step_desc* d, StepArgs& a, int dtype);
// Validate the tiles (each inside its set, disjoint within a set) and
// count chunks per stream.  `idx` is host scratch of n_tiles entries, used
// only when a set's tiles are not in increasing order.  No allocation.
int32_t plan_chunks(const StepArgs& a, const int64_t* tiles, int32_t n_tiles, int32_t* idx, ChunkPlan& plan);
ChunkBuildArgs chunk_build_args(const StepArgs& a, const ChunkPlan& plan);
}  // namespace qedmi
