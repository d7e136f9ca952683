// qed_step_noalloc: the fused step for callers that cannot allocate device
// memory (code under graph capture, serving loops, allocator-free
// harnesses).  Its scratch is one file-scope device array per GPU:
//
//   [0, 256)             chunk ticket (monotonic, cleared once at set-up)
//   status words         one 64-bit look-back word per chunk (epoch-tagged,
//                        so they never need clearing between calls)
//   chunk table          rebuilt on the device by every call
//   tile list            copied through kernel arguments by every call
//   builder scratch      order / first-chunk arrays of the chunk builder
//
// The host side takes the array's device address with hipGetSymbolAddress
// once per device and uses only that address afterwards.  Every call on a
// device shares the array: calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace qedmi {
namespace {

constexpr int kStaticMaxChunks = 65536;   // 2^28 particles in chunks of 4096
constexpr int kStaticMaxTiles = 8192;
constexpr size_t kOffStatus = 256;
constexpr size_t kOffChunks = kOffStatus + sizeof(unsigned long long) * kStaticMaxChunks;
constexpr size_t kOffTiles = kOffChunks + sizeof(ChunkDesc) * kStaticMaxChunks;
constexpr size_t kOffPart = kOffTiles + 3 * sizeof(int64_t) * kStaticMaxTiles;
constexpr size_t kScratchBytes = kOffPart + 2 * sizeof(int32_t) * kStaticMaxTiles;   // 2.81 MiB
static_assert(kOffChunks % 256 == 0 && kOffTiles % 256 == 0 && kOffPart % 256 == 0, "aligned regions");

}  // namespace
}  // namespace qedmi

static __device__ __align__(256) unsigned char scratch[qedmi::kScratchBytes];

namespace qedmi {
namespace {

constexpr int kMaxDevices = 64;
constexpr int kGridSlots = 8;

struct DeviceState {
    unsigned char* ptr = nullptr;            // device address of `scratch` on this device
    unsigned long long ticket_issued = 0;    // host mirror of the ticket counter
    uint32_t epoch = 0;
    struct {
        int dtype, surr, chi_mode;
        size_t lds;
        int grid;
    } grids[kGridSlots];
    int n_grids = 0;
};

DeviceState g_state[kMaxDevices];
std::mutex g_setup;

__global__ void __launch_bounds__(256) clear_words(unsigned long long* p, int64_t n) {
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += gridDim.x * 256LL) p[i] = 0ULL;
}

int32_t fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return QED_ERR_HIP;
}

// First call on a device: the array's address on this device, and the
// ticket and status words cleared (on the caller's stream, ahead of the
// step that follows).
int32_t setup(int dev, hipStream_t s, DeviceState** out) {
    std::lock_guard<std::mutex> lock(g_setup);
    DeviceState& st = g_state[dev];
    if (!st.ptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail(e, "address of the static scratch");
        const int64_t words = static_cast<int64_t>(kOffChunks / sizeof(unsigned long long));
        hipLaunchKernelGGL(clear_words, dim3(64), dim3(256), 0, s, static_cast<unsigned long long*>(p), words);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(e, "static scratch clear");
        st.ptr = static_cast<unsigned char*>(p);
        st.ticket_issued = 0;
        st.epoch = 0;
    }
    *out = &st;
    return QED_OK;
}

int grid_for(DeviceState& st, const StepArgs& a, int dtype, int dev) {
    const int surr = (a.use_bw_surr || a.use_qs_surr) ? 1 : 0;
    const size_t lds = step_lds_bytes_for(a, dtype);
    for (int i = 0; i < st.n_grids; ++i)
        if (st.grids[i].dtype == dtype && st.grids[i].surr == surr && st.grids[i].chi_mode == a.chi_mode &&
            st.grids[i].lds == lds)
            return st.grids[i].grid;
    const int grid = step_grid_size(a, dtype, dev);
    if (st.n_grids < kGridSlots) st.grids[st.n_grids++] = {dtype, surr, a.chi_mode, lds, grid};
    return grid;
}

}  // namespace
}  // namespace qedmi

using namespace qedmi;

extern "C" int32_t qed_step_noalloc(const qed_context* ctx, const qed_step_desc* d, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every argument check comes before the first HIP call
    StepArgs a;
    int dtype = 0;
    int32_t r = prepare_sets(d, false, a, dtype);
    if (r) return r;
    const int64_t* tiles = d->n_tiles > 0 ? d->tiles : nullptr;
    if (tiles && d->n_tiles > kStaticMaxTiles) {
        set_error("qed_step_noalloc takes at most 8192 tiles");
        return QED_ERR_INVALID;
    }
    int32_t idx[kStaticMaxTiles];   // host scratch of the overlap check (stack)
    ChunkPlan plan;
    r = plan_chunks(a, tiles, d->n_tiles, idx, plan);
    if (r) return r;
    if (plan.n_chunks > kStaticMaxChunks) {
        set_error("qed_step_noalloc takes at most 65536 chunks of 4096 particles (2^28 particles)");
        return QED_ERR_INVALID;
    }
    r = prepare_tables(ctx ? ctx->units : Units{}, d, a, dtype);
    if (r) return r;
    if (plan.n_chunks == 0) return QED_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) { set_error("device index beyond 63"); return QED_ERR_INVALID; }
    if (ctx && ctx->device != dev) { set_error("context belongs to another device"); return QED_ERR_INVALID; }
    DeviceState* st = nullptr;
    r = setup(dev, s, &st);
    if (r) return r;
    unsigned char* base = st->ptr;
    int64_t* d_tiles = reinterpret_cast<int64_t*>(base + kOffTiles);
    if (tiles) {
        e = store_tiles_by_args(tiles, d->n_tiles, d_tiles, s);
        if (e != hipSuccess) return fail(e, "tile list upload");
    }
    ChunkBuildArgs b = chunk_build_args(a, plan);
    b.tiles = tiles ? d_tiles : nullptr;
    b.order = reinterpret_cast<int32_t*>(base + kOffPart);
    b.ostart = b.order + kStaticMaxTiles;
    b.chunks = reinterpret_cast<ChunkDesc*>(base + kOffChunks);
    e = launch_chunk_build(b, s);
    if (e != hipSuccess) return fail(e, "chunk table build");
    a.n_chunks = plan.n_chunks;
    const int grid = std::max(1, std::min(a.n_chunks, grid_for(*st, a, dtype, dev)));
    st->epoch = st->epoch + 1 == 0 ? 1 : st->epoch + 1;
    a.status = reinterpret_cast<unsigned long long*>(base + kOffStatus);
    a.ticket = reinterpret_cast<unsigned long long*>(base);
    a.ticket_base = st->ticket_issued;
    a.epoch = st->epoch;
    a.chunks = b.chunks;
    e = launch_step(a, dtype, grid, s);
    if (e != hipSuccess) return fail(e, "step launch");
    // every block takes exactly one failing ticket before it exits
    st->ticket_issued += static_cast<unsigned long long>(a.n_chunks) + static_cast<unsigned long long>(grid);
    return QED_OK;
}
