// Chunk table of the fused step, built on the device from the tile list.
//
// The fused step hands out chunks of at most kChunk consecutive particles
// of one tile, ordered by product stream (leptons, then photons) and,
// within a stream, by tile order; products are appended in that order.
// Building the table on the device keeps the host out of the step: the
// host validates the tiles and counts chunks (O(tiles)), then two kernels
// place every tile in its stream (one block, prefix over tiles) and write
// every chunk (one thread per chunk, binary search over the tiles' first
// chunk indices).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace qedmi {

namespace {

constexpr int kPrefixThreads = 1024;

struct TileView {
    int64_t set, begin, end;
};

__device__ __forceinline__ TileView tile_at(const ChunkBuildArgs& a, int t) {
    if (a.tiles) return {a.tiles[3 * t], a.tiles[3 * t + 1], a.tiles[3 * t + 2]};
    return {t, 0, a.set_n[t]};   // one tile per set
}

// Inclusive block-wide sum of four counters at once (wave shuffles, then
// one LDS round over the waves).
__device__ __forceinline__ int4 block_scan4(int4 v, int4* s_wave) {
    const int lane = static_cast<int>(__lane_id());
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int x = __shfl_up(v.x, o), y = __shfl_up(v.y, o), z = __shfl_up(v.z, o), w = __shfl_up(v.w, o);
        if (lane >= o) {
            v.x += x;
            v.y += y;
            v.z += z;
            v.w += w;
        }
    }
    if (lane == 63) s_wave[wave] = v;
    __syncthreads();
    int4 off = make_int4(0, 0, 0, 0);
    for (int w = 0; w < wave; ++w) {
        off.x += s_wave[w].x;
        off.y += s_wave[w].y;
        off.z += s_wave[w].z;
        off.w += s_wave[w].w;
    }
    __syncthreads();
    return make_int4(v.x + off.x, v.y + off.y, v.z + off.z, v.w + off.w);
}

// One block: every tile with at least one chunk gets its position among the
// stream's tiles (stream 0 first, then stream 1, each in tile order) and the
// index of its first chunk.
__global__ void __launch_bounds__(kPrefixThreads) chunk_prefix_kernel(ChunkBuildArgs a) {
    __shared__ int4 s_wave[kPrefixThreads / 64];
    __shared__ int4 s_carry;
    if (threadIdx.x == 0) s_carry = make_int4(0, 0, 0, 0);
    __syncthreads();
    for (int t0 = 0; t0 < a.n_tiles; t0 += kPrefixThreads) {
        const int t = t0 + static_cast<int>(threadIdx.x);
        int stream = -1, cnt = 0;
        if (t < a.n_tiles) {
            const TileView tv = tile_at(a, t);
            stream = a.set_stream[tv.set];
            const int64_t len = tv.end - tv.begin;
            cnt = (stream >= 0 && len > 0) ? static_cast<int>((len + kChunk - 1) / kChunk) : 0;
            if (cnt == 0) stream = -1;
        }
        // (tiles of stream 0, chunks of stream 0, tiles of stream 1, chunks of stream 1)
        const int4 mine = make_int4(stream == 0, stream == 0 ? cnt : 0, stream == 1, stream == 1 ? cnt : 0);
        const int4 carry = s_carry;
        const int4 incl = block_scan4(mine, s_wave);
        if (stream == 0) {
            const int pos = carry.x + incl.x - 1;
            a.order[pos] = t;
            a.ostart[pos] = carry.y + incl.y - cnt;
        } else if (stream == 1) {
            const int pos = a.n_part0 + carry.z + incl.z - 1;
            a.order[pos] = t;
            a.ostart[pos] = a.n_chunks0 + carry.w + incl.w - cnt;
        }
        __syncthreads();
        if (threadIdx.x == kPrefixThreads - 1)
            s_carry = make_int4(carry.x + incl.x, carry.y + incl.y, carry.z + incl.z, carry.w + incl.w);
        __syncthreads();
    }
}

// One thread per chunk: the last placed tile whose first chunk is <= k.
__global__ void __launch_bounds__(256) chunk_fill_kernel(ChunkBuildArgs a) {
    const int k = blockIdx.x * 256 + static_cast<int>(threadIdx.x);
    if (k >= a.n_chunks) return;
    int lo = 0, hi = a.n_part;   // invariant: ostart[lo] <= k < ostart[hi] (ostart[n_part] = n_chunks)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.ostart[mid] <= k) lo = mid;
        else hi = mid;
    }
    const TileView tv = tile_at(a, a.order[lo]);
    const int stream = a.set_stream[tv.set];
    ChunkDesc c{};
    c.begin = tv.begin + static_cast<int64_t>(k - a.ostart[lo]) * kChunk;
    c.set = static_cast<int32_t>(tv.set);
    c.len = static_cast<int32_t>(tv.end - c.begin < kChunk ? tv.end - c.begin : kChunk);
    c.stream = stream;
    c.stream_first = stream == 0 ? 0 : a.n_chunks0;
    c.stream_last = stream == 0 ? a.n_chunks0 - 1 : a.n_chunks - 1;
    a.chunks[k] = c;
}

// Tiles carried in the kernel arguments (for callers that have no pinned
// staging memory): up to kTilesPerBatch triples per launch.
constexpr int kTilesPerBatch = 160;
struct TileBatch {
    int32_t first, n;
    int64_t v[3 * kTilesPerBatch];
};

__global__ void __launch_bounds__(256) tile_store_kernel(TileBatch b, int64_t* dst) {
    for (int i = threadIdx.x; i < 3 * b.n; i += 256) dst[3 * static_cast<int64_t>(b.first) + i] = b.v[i];
}

}  // namespace

hipError_t launch_chunk_build(const ChunkBuildArgs& a, hipStream_t s) {
    if (a.n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(chunk_prefix_kernel, dim3(1), dim3(kPrefixThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(chunk_fill_kernel, dim3((a.n_chunks + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t store_tiles_by_args(const int64_t* host_tiles, int n_tiles, int64_t* dst, hipStream_t s) {
    for (int t0 = 0; t0 < n_tiles; t0 += kTilesPerBatch) {
        TileBatch b;
        b.first = t0;
        b.n = n_tiles - t0 < kTilesPerBatch ? n_tiles - t0 : kTilesPerBatch;
        for (int i = 0; i < 3 * b.n; ++i) b.v[i] = host_tiles[3 * static_cast<int64_t>(t0) + i];
        hipLaunchKernelGGL(tile_store_kernel, dim3(1), dim3(256), 0, s, b, dst);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace qedmi
