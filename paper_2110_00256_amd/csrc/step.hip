// HIP kernels of the QED sub-step for gfx950 (MI355X).
//
// step_kernel: one persistent launch processes chunks of kChunk particles
// taken from an atomic ticket counter.  For each chunk:
//   stream   each wave streams its own quarter of the chunk's particle SoA
//            (coalesced), computes chi, the total rate from the 1D table
//            staged in LDS, tau <- tau - rate dt and the event predicate
//            tau < 0 (paper Fig. 1, Sec. 3), and appends its events' chunk
//            positions, in order, to its own region of an LDS list (ballot,
//            mbcnt, running count); the events' chi goes to LDS;
//   counts   one barrier: the four waves' counts give the chunk's event
//            total, published at once for the decoupled look-back
//            (Merrill & Garland 2016); tickets are taken in chunk order, so
//            every predecessor is already running;
//   events   dense rounds over the chunk's events, one per thread: Philox
//            draws, inverse-CDF sample (table, or the MLP surrogate on the
//            round's 64 events of a wave), product kinematics (Sec. 2.1,
//            2.2), parent update; after the first round the block resolves
//            the exclusive prefix over earlier chunks of the same product
//            stream, and products go to deterministic slots in parent order.
#include <hip/hip_runtime.h>

#include "device_physics.hpp"
#include "internal.hpp"
#include "surrogate.hpp"

namespace qedmi {

namespace {

constexpr unsigned kFlagA = 1u, kFlagP = 2u;
constexpr unsigned long long kValueMask = (1ULL << kStatusBits) - 1ULL;
constexpr int kSpinLimit = 1 << 24;

__device__ __forceinline__ unsigned long long pack_status(uint32_t epoch, unsigned flag,
                                                          unsigned long long v) {
    return (static_cast<unsigned long long>(epoch) << 32) | (static_cast<unsigned long long>(flag) << 30) |
           (v & kValueMask);
}

template <typename T>
__device__ __forceinline__ T ld(const void* p, int64_t i) {
    return static_cast<const T*>(p)[i];
}
template <typename T>
__device__ __forceinline__ void st(void* p, int64_t i, T v) {
    static_cast<T*>(p)[i] = v;
}
// Streaming (non-temporal) stores for values written once per step and not
// read again in it (optical depths, parent updates, products), so that they
// do not evict the lookup tables the inverse-CDF search walks from L2.
template <typename T>
__device__ __forceinline__ void stnt(void* p, int64_t i, T v) {
    __builtin_nontemporal_store(v, static_cast<T*>(p) + i);
}

template <typename T>
__device__ __forceinline__ const T* ln_rate_ptr(const TableDev& t);
template <>
__device__ __forceinline__ const double* ln_rate_ptr<double>(const TableDev& t) { return t.ln_rate64; }
template <>
__device__ __forceinline__ const float* ln_rate_ptr<float>(const TableDev& t) { return t.ln_rate32; }

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ unsigned bits_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<unsigned>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<unsigned>(mask), 0u));
}

// Decoupled look-back (Merrill & Garland 2016), in two halves: publish()
// (one thread) posts the chunk's aggregate as soon as it is known, resolve()
// (one wave) later returns the exclusive prefix over earlier chunks of the
// same product stream and posts the inclusive one.  A status word carries
// the launch epoch, the flag and the value together, so relaxed
// device-scope atomics are enough: no other data is published through it.
// (Acquire/release at device scope would invalidate or write back the whole
// L2 of the XCD on every poll.)  The base counts read before phase 1
// complete before any aggregate is published: their values are in LDS.
__device__ __forceinline__ void publish(const StepArgs& a, int k, const ChunkDesc& c, unsigned long long agg) {
    __hip_atomic_store(a.status + k, pack_status(a.epoch, k == c.stream_first ? kFlagP : kFlagA, agg),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// resolve() is called by the whole block: thread t polls chunk base - t, so
// a window of kBlock predecessors costs one round of loads (with many
// chunks in flight the nearest inclusive prefix can lie hundreds of chunks
// back).  The nearest predecessor holding an inclusive prefix (flag P) ends
// the walk; every chunk between it and k must have posted at least its
// aggregate, else the window is polled again.  Chunks before the stream's
// first count as P with value 0.  Returns the exclusive prefix in every
// thread; thread 0 posts the inclusive one.  `s_p` and `s_sum` are LDS
// scratch of one entry per wave.
__device__ long long resolve(const StepArgs& a, int k, const ChunkDesc& c, unsigned long long agg, int64_t* err,
                             int* s_p, long long* s_sum) {
    const int tid = threadIdx.x, wave = tid >> 6;
    const int lane = static_cast<int>(lane_id());
    long long excl = 0;
    if (k != c.stream_first) {
        int base = k - 1;
        int spins = 0;
        for (;;) {
            const int j = base - tid;
            unsigned flag = kFlagP;
            long long val = 0;
            if (j >= c.stream_first) {
                const unsigned long long v = __hip_atomic_load(a.status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                flag = static_cast<uint32_t>(v >> 32) == a.epoch ? (static_cast<unsigned>(v >> 30) & 3u) : 0u;
                val = static_cast<long long>(v & kValueMask);
            }
            const unsigned long long pmask = __ballot(flag == kFlagP);
            if (lane == 0) s_p[wave] = pmask ? wave * 64 + __builtin_ctzll(pmask) : kBlock;
            __syncthreads();
            int p = kBlock;   // nearest P in the window, kBlock: none
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) p = min(p, s_p[w]);
            // a chunk on the way has not posted: poll the window again
            if (__syncthreads_or(flag == 0u && tid <= p)) {
                if (++spins > kSpinLimit) {   // predecessor never published: give up, report
                    if (err && tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(err), 1ULL);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            long long part = tid <= p ? val : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
            if (lane == 0) s_sum[wave] = part;
            __syncthreads();
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) excl += s_sum[w];
            __syncthreads();   // s_p and s_sum are reused by the next round
            if (p < kBlock) break;
            base -= kBlock;
        }
    }
    if (tid == 0)
        __hip_atomic_store(a.status + k, pack_status(a.epoch, kFlagP, static_cast<unsigned long long>(excl) + agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// Products, like the parents' updates, are written once and not read again
// in the step: non-temporal stores keep them from displacing the tables and
// the events' gathered u and w in L2.
template <typename T>
__device__ __forceinline__ void write_product(const AppendDev& o, int64_t slot, T ux, T uy, T uz, T w, T tau,
                                              int64_t parent) {
    if (slot >= o.capacity) return;
    stnt<T>(o.ux, slot, ux);
    stnt<T>(o.uy, slot, uy);
    stnt<T>(o.uz, slot, uz);
    stnt<T>(o.w, slot, w);
    stnt<T>(o.tau, slot, tau);
    if (o.parent) __builtin_nontemporal_store(static_cast<long long>(parent),
                                              reinterpret_cast<long long*>(o.parent) + slot);
}

// Surrogate sampling for the events of one wave (all 64 lanes call it
// together; `valid` marks lanes holding an event).  Lanes outside the
// trained domain use the table.  When `probe` is set (wave-uniform) one
// lane also evaluates the table and, if the network is off by more than
// probe_tol in its output space, the whole wave falls back to the table and
// `failed` is set.  Returns the network-side sample (QS: ln xi; BW: xi), or
// NAN where the caller must use the table; `batch` tells whether the
// network ran for this wave.
__device__ __forceinline__ float surr_wave_sample(const SurrogateDev& sv, const SurrLds* lw, const TableDev& tab,
                                                  bool valid, float chi, float u, bool probe, bool& batch,
                                                  bool& failed) {
    float x0 = 0.f, x1 = 0.f;
    const bool inside = valid && surr_inputs(sv, chi, u, x0, x1);
    const unsigned long long in_mask = __ballot(inside);
    batch = in_mask != 0ULL;
    failed = false;
    if (!batch) return __builtin_nanf("");
    const float y = surr_forward_wave_lds(lw, x0, x1);
    if (!probe) return inside ? surr_output(sv, chi, u, y) : __builtin_nanf("");
    // probe: the first lane with an in-domain event
    const unsigned probe_lane = static_cast<unsigned>(__builtin_ctzll(in_mask));
    float err = 0.f;
    if (__lane_id() == probe_lane) {
        float ref;
        if (sv.process == 1) {
            ref = dev::sample_qs_lnxi<float>(tab, chi, u);
        } else {
            bool e;
            ref = dev::sample_bw<float>(tab, chi, u, e);
        }
        err = fabsf(y - surr_target_of(sv.process, chi, u, ref));
    }
    err = __shfl(err, static_cast<int>(probe_lane));
    failed = !(err <= sv.probe_tol);
    if (failed || !inside) return __builtin_nanf("");
    return surr_output(sv, chi, u, y);
}

// Classical radiation below the QED threshold (Sec. 6): the energy
// radiated classically, (2/3)(alpha m c^2/hbar) chi^2 dt in m c^2 (`drag`
// holds the factor in front of chi^2), is taken from the particle along its
// direction of motion: gamma' = max(1, gamma - dgamma), u' = u
// sqrt(gamma'^2 - 1)/|u|.
template <typename T>
__device__ __forceinline__ void classical_drag(const SetDev& S, int64_t j, T ux, T uy, T uz, T chi, double drag,
                                               double inv_u) {
    const double x = ux, y = uy, z = uz;
    const double u2 = x * x + y * y + z * z;
    if (!(u2 > 0.0)) return;
    const double c = chi;
    const double gp = sqrt(1.0 + u2) - drag * c * c;
    const double sc = gp > 1.0 ? sqrt((gp - 1.0) * (gp + 1.0)) / sqrt(u2) : 0.0;
    st<T>(S.p[0], j, static_cast<T>(x * sc * inv_u));
    st<T>(S.p[1], j, static_cast<T>(y * sc * inv_u));
    st<T>(S.p[2], j, static_cast<T>(z * sc * inv_u));
}

template <typename T, int kChiMode, bool kSurr>
__device__ __forceinline__ void step_body(const StepArgs& a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nbw = a.bw.n_chi > 0 ? a.bw.n_chi : 0;
    const int nqs = a.qs.n_chi > 0 ? a.qs.n_chi : 0;
    T* t_bw = reinterpret_cast<T*>(lds_raw);
    T* t_qs = t_bw + ((nbw + 1) & ~1);
    // event lists: wave w owns chunk positions [w kWaveSpan, (w + 1) kWaveSpan)
    // and appends the positions of its events, in order, to its own region
    uint16_t* evlist = reinterpret_cast<uint16_t*>(t_qs + ((nqs + 1) & ~1));
    // chi of the chunk's event particles at their chunk index (written while
    // streaming), then their sample (BW xi, QS xi)
    T* s_chi = reinterpret_cast<T*>(evlist + kChunk);
    // surrogate path: the weights of the process whose chunk is in hand
    SurrLds* s_net = reinterpret_cast<SurrLds*>(
        lds_raw + ((reinterpret_cast<unsigned char*>(s_chi + kChunk) - lds_raw + 15) & ~static_cast<ptrdiff_t>(15)));
    int staged = -1;
    __shared__ unsigned long long kmask[kMasks];
    __shared__ int kpref[kMasks];
    __shared__ int s_wcnt[kBlock / 64];
    __shared__ int s_lbp[kBlock / 64];          // look-back scratch
    __shared__ long long s_lbsum[kBlock / 64];
    __shared__ int s_ticket, s_kept;
    __shared__ long long s_excl, s_base0, s_base1;

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const unsigned lane = lane_id();

    if (a.bw.ln_rate64 || a.bw.ln_rate32)
        for (int i = tid; i < nbw; i += kBlock) t_bw[i] = ln_rate_ptr<T>(a.bw)[i];
    if (a.qs.ln_rate64 || a.qs.ln_rate32)
        for (int i = tid; i < nqs; i += kBlock) t_qs[i] = ln_rate_ptr<T>(a.qs)[i];

    // launch statistics, accumulated per block and added once at the end
    // (one atomic per counter and block instead of one per chunk or batch)
    unsigned long long n_updates = 0, n_qs_events = 0, n_bw_events = 0, n_kept = 0;
    unsigned long long n_surr_batches = 0, n_surr_fallbacks = 0;   // lane 0 of each wave
    unsigned n_nonfinite = 0;   // per thread: chi not finite, or tau NaN or -inf

    // A ticket is drawn only when the block is free to start the chunk: a
    // chunk drawn ahead would start late, and its successors, already
    // running, would wait for it in their look-back (measured 8% slower).
    for (;;) {
        __syncthreads();
        if (tid == 0) s_ticket = static_cast<int>(atomicAdd(a.ticket, 1ULL) - a.ticket_base);
        __syncthreads();
        const int k = s_ticket;
        if (k >= a.n_chunks) break;
        const ChunkDesc c = a.chunks[k];
        const SetDev& S = a.sets[c.set];
        const bool photon = (c.stream == 1);
        if (tid == 0) {
            if (photon) {
                s_base0 = *a.el.count;
                s_base1 = *a.po.count;
            } else {
                s_base0 = *a.ph.count;
                s_base1 = 0;
            }
        }

        // ---------------- phase 1: stream, evolve, flag
        const T dt = dev::par<T>(a.dt, a.dt_f);
        // each wave streams its own contiguous quarter of the chunk and
        // appends its events (chunk positions, in order) to its region of
        // evlist with a running count: no block-wide list pass is needed
        constexpr int kWaveSpan = kChunk / (kBlock / 64);
        const int wbase = wave * kWaveSpan;
        int wcnt = 0;
        if (a.generate_only) {
            // The flags of all the wave's slices are loaded together (one
            // round trip), then the flagged particles' fields slice by slice,
            // the next slice's loads issued before the current slice is
            // evaluated (the loop is unrolled, so no copy waits for them).
            // Lanes past the end read the chunk's first flag and drop it.
            // FP32: the field loads are not predicated on the flag (lanes
            // without a flagged particle read the slice's first particle,
            // a line the wave reads anyway or one more line per array):
            // loads under a branch make the compiler wait for every load in
            // flight before the next use, which undoes the overlap.  With
            // every particle flagged this took the FP32 production calls of
            // 1e8 particles from 6.2 to 4.2 ms; FP64 keeps the predicated
            // loads (6.5 / 6.1 ms against 6.3 / 6.7 ms unpredicated).
            constexpr int kSlices = kWaveSpan / 64;
            uint8_t fl[kSlices];
#pragma unroll
            for (int sl = 0; sl < kSlices; ++sl) {
                const int loc = wbase + sl * 64 + static_cast<int>(lane);
                fl[sl] = S.flags[c.begin + (loc < c.len ? loc : 0)];
            }
            unsigned fmask = 0;   // bit sl: this lane's particle of slice sl is flagged
#pragma unroll
            for (int sl = 0; sl < kSlices; ++sl)
                if (fl[sl] != 0 && wbase + sl * 64 + static_cast<int>(lane) < c.len) fmask |= 1u << sl;
            auto load_fields = [&](int sl, T (&f)[9]) {
                const int loc = wbase + sl * 64 + static_cast<int>(lane);
                if constexpr (sizeof(T) == 4) {
                    const int first = wbase + sl * 64 < c.len ? wbase + sl * 64 : 0;
                    const int64_t j = c.begin + (((fmask >> sl) & 1u) ? loc : first);
#pragma unroll
                    for (int q = 0; q < 9; ++q) f[q] = ld<T>(S.p[q], j);
                } else if ((fmask >> sl) & 1u) {
                    const int64_t j = c.begin + loc;
#pragma unroll
                    for (int q = 0; q < 9; ++q) f[q] = ld<T>(S.p[q], j);
                }
            };
            const T su = dev::par<T>(a.units.u, a.units.u_f), se = dev::par<T>(a.units.e, a.units.e_f),
                    sb = dev::par<T>(a.units.b, a.units.b_f);
            T cur[9] = {}, nxt[9] = {};
            load_fields(0, cur);
#pragma unroll
            for (int sl = 0; sl < kSlices; ++sl) {
                if (sl + 1 < kSlices) load_fields(sl + 1, nxt);
                const int loc = wbase + sl * 64 + static_cast<int>(lane);
                const bool ev = (fmask >> sl) & 1u;
                if (ev) {
                    const T ux = su * cur[0], uy = su * cur[1], uz = su * cur[2];
                    const T ex = se * cur[3], ey = se * cur[4], ez = se * cur[5];
                    const T bx = sb * cur[6], by = sb * cur[7], bz = sb * cur[8];
                    s_chi[loc] = photon
                        ? static_cast<T>(dev::chi_of<T, true>(kChiMode, ux, uy, uz, ex, ey, ez, bx, by, bz).chi)
                        : static_cast<T>(dev::chi_of<T, false>(kChiMode, ux, uy, uz, ex, ey, ez, bx, by, bz).chi);
                }
                const unsigned long long m = __ballot(ev);
                if (ev) evlist[wbase + wcnt + static_cast<int>(bits_below(m))] = static_cast<uint16_t>(loc);
                wcnt += __popcll(m);
#pragma unroll
                for (int q = 0; q < 9; ++q) cur[q] = nxt[q];
            }
        } else {
            // FP64: one particle per lane at a time, the next one's ten
            // loads issued before the current one is evaluated (stores in
            // between could alias them, so the compiler would not hoist the
            // loads itself); FP32: four particles' loads issued together, two
            // in the surrogate kernel (whose network pass leaves fewer
            // registers to the stream: with four, values live across the
            // chunk were spilled and reloaded inside this loop).
            // Lanes past the end load the chunk's first particle and drop it.
            constexpr bool kPipe = sizeof(T) == 8;
            constexpr int kBatch = sizeof(T) == 8 ? 1 : (kSurr ? 2 : 4);
            constexpr int kIters = kWaveSpan / 64;
            static_assert(kIters % kBatch == 0, "a wave's span must be a whole number of batches");
            auto load_batch = [&](int it, T (&v)[kBatch][10]) {
#pragma unroll
                for (int b = 0; b < kBatch; ++b) {
                    const int loc = wbase + (it + b) * 64 + static_cast<int>(lane);
                    const int64_t j = c.begin + (loc < c.len ? loc : 0);
                    // ordinary loads for all ten arrays: non-temporal loads
                    // for the fields and tau (read once) measured the same
                    // for the table kernels and 20% slower for the
                    // surrogate kernel
#pragma unroll
                    for (int q = 0; q < 10; ++q) v[b][q] = ld<T>(S.p[q], j);
                }
            };
            auto eval_batch = [&](int it, T (&v)[kBatch][10]) {
#pragma unroll
                for (int b = 0; b < kBatch; ++b) {
                    // caller units -> u = p/(m_e c), V/m, T (factors 1 for SI)
#pragma unroll
                    for (int q = 0; q < 9; ++q)
                        v[b][q] *= q < 3 ? dev::par<T>(a.units.u, a.units.u_f)
                                         : q < 6 ? dev::par<T>(a.units.e, a.units.e_f) : dev::par<T>(a.units.b, a.units.b_f);
                    const int loc = wbase + (it + b) * 64 + static_cast<int>(lane);
                    bool ev = false;
                    if (loc < c.len) {
                        const int64_t j = c.begin + loc;
                        T rate, chi;
                        if (photon) {
                            const dev::ChiGamma cg = dev::chi_of<T, true>(kChiMode, v[b][0], v[b][1], v[b][2], v[b][3],
                                                                          v[b][4], v[b][5], v[b][6], v[b][7], v[b][8]);
                            chi = static_cast<T>(cg.chi);
                            rate = dev::rate_bw<T>(t_bw, a.bw, chi, static_cast<T>(cg.gamma));
                        } else {
                            const dev::ChiGamma cg = dev::chi_of<T, false>(kChiMode, v[b][0], v[b][1], v[b][2], v[b][3],
                                                                           v[b][4], v[b][5], v[b][6], v[b][7], v[b][8]);
                            chi = static_cast<T>(cg.chi);
                            rate = dev::rate_qs<T>(t_qs, a.qs, chi, static_cast<T>(cg.gamma));
                        }
                        T tn = v[b][9] - rate * dt;
                        ev = tn < T(0);
                        if (a.chi_qed_min > 0.0 && static_cast<double>(chi) < a.chi_qed_min) {
                            // classical regime: tau is kept, leptons radiate classically
                            ev = false;
                            tn = v[b][9];
                            if (!photon)
                                classical_drag<T>(S, j, v[b][0], v[b][1], v[b][2], chi, a.drag, a.units.inv_u);
                        }
                        // +inf is a decayed photon's optical depth, not an error
                        constexpr T kBig = sizeof(T) == 8 ? T(1.7976931348623157e308) : T(3.40282347e38f);
                        n_nonfinite += !(chi <= kBig) || !(tn >= -kBig);
                        if (ev) s_chi[loc] = chi;
                        else stnt<T>(S.p[9], j, tn);
                        if (S.flags) S.flags[j] = static_cast<uint8_t>(ev);
                    }
                    const unsigned long long m = __ballot(ev);
                    if (ev) evlist[wbase + wcnt + static_cast<int>(bits_below(m))] = static_cast<uint16_t>(loc);
                    wcnt += __popcll(m);
                }
            };
            if constexpr (kPipe) {
                T v[kBatch][10], w[kBatch][10];
                load_batch(0, v);
                for (int it = 0; it < kIters; it += kBatch) {
                    if (it + kBatch < kIters) load_batch(it + kBatch, w);
                    eval_batch(it, v);
#pragma unroll
                    for (int b = 0; b < kBatch; ++b)
#pragma unroll
                        for (int q = 0; q < 10; ++q) v[b][q] = w[b][q];
                }
            } else {
                for (int it = 0; it < kIters; it += kBatch) {
                    T v[kBatch][10];
                    load_batch(it, v);
                    eval_batch(it, v);
                }
            }
        }
        // ---------------- the chunk's events in order: wave w's region first
        // (wave-major order is particle order); event e lives in the region
        // of the wave whose prefix range holds it
        if (lane == 0) s_wcnt[wave] = wcnt;
        __syncthreads();
        const int p1 = s_wcnt[0], p2 = p1 + s_wcnt[1], p3 = p2 + s_wcnt[2];
        const int total = p3 + s_wcnt[3];
        auto ev_loc = [&](int e) -> int {
            const int w = (e >= p1) + (e >= p2) + (e >= p3);
            const int pw = w == 0 ? 0 : w == 1 ? p1 : w == 2 ? p2 : p3;
            return evlist[w * kWaveSpan + e - pw];
        };

        // ---------------- surrogate (FP32 data only): the network runs inside
        // the event rounds, each wave over its 64 events of the round, on the
        // round's own draw; its weights are staged in LDS once per block and
        // process.  Events outside its served domain, and those of a wave
        // whose probe failed earlier in the chunk, use the table.
        bool surr_on = false;
        bool surr_failed = false;
        if constexpr (kSurr && sizeof(T) == 4) {
            surr_on = photon ? a.use_bw_surr : a.use_qs_surr;
            if (surr_on && staged != static_cast<int>(photon)) {
                surr_stage(photon ? a.bw_surr : a.qs_surr, s_net, tid, kBlock);
                staged = static_cast<int>(photon);
                __syncthreads();
            }
        }
        // the network's sample for this lane's event (QS: ln xi, BW: xi), NaN
        // where the table samples; called by every lane of the wave
        auto net_sample = [&](bool valid, T cs, double u0, int round) -> float {
            if constexpr (kSurr && sizeof(T) == 4) {
                if (!surr_on) return __builtin_nanf("");
                const SurrogateDev& sv = photon ? a.bw_surr : a.qs_surr;
                const bool probe = ((k + wave + round) % sv.probe_every) == 0;
                bool batch, failed;
                float v = surr_wave_sample(sv, s_net, photon ? a.bw : a.qs, valid, static_cast<float>(cs),
                                           static_cast<float>(u0), probe, batch, failed);
                surr_failed = surr_failed || failed;
                if (surr_failed) v = __builtin_nanf("");
                if (lane == 0 && batch) {
                    ++n_surr_batches;
                    if (surr_failed) ++n_surr_fallbacks;
                }
                return v;
            } else {
                return __builtin_nanf("");
            }
        };

        // ---------------- events.  Per event: the draws (Philox block 0 of
        // the parent), the inverse-CDF sample (table search on chi, or the
        // surrogate network inside its served bands), the kinematics, the parent's new
        // u and tau, and the products at deterministic slots in parent order:
        // slot = exclusive prefix of the stream's product counts over earlier
        // chunks (decoupled look-back) + the event's rank in this chunk.
        const bool thresh = !photon && a.photon_min_energy > 0.0;
        const T su = dev::par<T>(a.units.u, a.units.u_f), iu = dev::par<T>(a.units.inv_u, a.units.inv_u_f);
        // sample of event e from its chi (or surrogate sample) `cs` and u0
        auto sample_of = [&](bool have, T cs, double u0) -> T {
            if (photon) {
                bool esel;
                const T rf = dev::bw_folded_uniform<T>(u0, esel);
                return have ? cs : dev::sample_bw_folded<T>(a.bw, cs, rf);
            }
            const T lr = dev::qs_log_uniform<T>(u0);
            return dev::dexp(have ? cs : dev::sample_qs_lnxi_lr<T>(a.qs, cs, lr));
        };
        int prods = total;
        if (!thresh) {
            // One dense pass.  The chunk's product count is the event count:
            // it is published at once.  The first round of events is drawn,
            // sampled and its parents updated before the block resolves the
            // prefix (giving the predecessors time to post theirs); products
            // are written from then on.
            if (tid == 0) publish(a, k, c, static_cast<unsigned long long>(total));
            long long excl = 0;   // the same in every thread once resolved
            // Each round's events' u and w are gathered at the top of the
            // round and scaled only after the draws (and the network), whose
            // arithmetic then covers the gathers' latency.  Loads complete in
            // issue order, so a value scaled as soon as it is gathered waits
            // for the gather where it is issued: gathering the next round's
            // events at the top of each round and scaling them there measured
            // 0.95 against 0.89 ms on the surrogate step and 3-4% slower
            // production calls.
#pragma unroll 1
            for (int e0 = 0, e = tid; e0 < total; e0 += kBlock, e += kBlock) {
                const bool valid = e < total;
                const int le = valid ? ev_loc(e) : 0;
                const int64_t j = c.begin + le;
                T rux = T(0), ruy = T(0), ruz = T(0), w = T(1);
                if (valid) {
                    rux = ld<T>(S.p[0], j);
                    ruy = ld<T>(S.p[1], j);
                    ruz = ld<T>(S.p[2], j);
                    if (S.p[10]) w = ld<T>(S.p[10], j);
                }
                const int64_t parent = S.id_base + j;
                const dev::Draws d = dev::draws<sizeof(T) == 4>(a.seed, static_cast<unsigned long long>(parent), a.step,
                                                static_cast<unsigned long long>(S.species), 0ULL);
                const T cs = valid ? s_chi[le] : T(1);
                const float nv = net_sample(valid, cs, d.u[0], e0 / kBlock);
                const bool have = valid && !__builtin_isnan(nv);
                const T xi = valid ? sample_of(have, have ? static_cast<T>(nv) : cs, d.u[0]) : T(0);
                // optical depths from uniforms 1 and 2: BW electron and
                // positron; QS parent (redrawn) and photon
                const T t1 = dev::neg_log_uniform<T>(d.u[1]);
                const T t2 = dev::neg_log_uniform<T>(d.u[2]);
                T ux, uy, uz;
                {
#pragma clang fp contract(off)
                    ux = su * rux;
                    uy = su * ruy;
                    uz = su * ruz;
                }
                T pa[3], pb[3];   // BW: the electron's and positron's u; QS: the photon's u
                if (photon) {
                    const bool esel = d.u[0] <= 0.5;   // on the 53-bit uniform, as the fold
                    const T sx = xi * ux * iu, sy = xi * uy * iu, sz = xi * uz * iu;
                    const T ox = ux * iu - sx, oy = uy * iu - sy, oz = uz * iu - sz;
                    pa[0] = esel ? sx : ox;
                    pa[1] = esel ? sy : oy;
                    pa[2] = esel ? sz : oz;
                    pb[0] = esel ? ox : sx;
                    pb[1] = esel ? oy : sy;
                    pb[2] = esel ? oz : sz;
                    if (valid) stnt<T>(S.p[9], j, static_cast<T>(__builtin_inf()));
                } else {
                    // QS photon energy gamma_gamma = (gamma - 1) xi, gamma - 1 = |u|^2/(gamma + 1)
                    const double dx = ux, dy = uy, dz = uz;
                    // FP64: the terms of |u|^2 in a fixed order, so that the
                    // results do not depend on how the compiler orders them
                    const double u2 = sizeof(T) == 8 ? fma(dz, dz, fma(dx, dx, dy * dy)) : dx * dx + dy * dy + dz * dz;
                    const T gg = static_cast<T>(u2 / (sqrt(1.0 + u2) + 1.0)) * xi;
                    const T um = static_cast<T>(sqrt(u2));
                    const T sc = um > T(0) ? gg / um : T(0);
                    const T px = sc * ux, py = sc * uy, pz = sc * uz;
                    pa[0] = px * iu;
                    pa[1] = py * iu;
                    pa[2] = pz * iu;
                    pb[0] = pb[1] = pb[2] = T(0);
                    if (valid) {
                        stnt<T>(S.p[0], j, (ux - px) * iu);
                        stnt<T>(S.p[1], j, (uy - py) * iu);
                        stnt<T>(S.p[2], j, (uz - pz) * iu);
                        stnt<T>(S.p[9], j, t1);
                    }
                }
                if (e0 == 0) {
                    excl = resolve(a, k, c, static_cast<unsigned long long>(total),
                                   a.stats ? a.stats + QED_STAT_SCAN_TIMEOUT : nullptr, s_lbp, s_lbsum);
                    if (tid == 0) s_excl = excl;
                }
                if (valid) {
                    const long long slot = excl + e;
                    if (photon) {
                        write_product<T>(a.el, s_base0 + slot, pa[0], pa[1], pa[2], w, t1, parent);
                        write_product<T>(a.po, s_base1 + slot, pb[0], pb[1], pb[2], w, t2, parent);
                    } else {
                        write_product<T>(a.ph, s_base0 + slot, pa[0], pa[1], pa[2], w, t2, parent);
                    }
                }
            }
            // a chunk without events adds nothing: its published aggregate
            // (0) lets later chunks look past it, and only a stream's last
            // chunk needs its prefix (for the stream's count)
            if (total == 0 && k == c.stream_last) {
                excl = resolve(a, k, c, 0ULL, a.stats ? a.stats + QED_STAT_SCAN_TIMEOUT : nullptr, s_lbp, s_lbsum);
                if (tid == 0) s_excl = excl;
            }
        } else {
            // With a photon threshold the chunk's product count is known only
            // after sampling: sample every event (no particle data needed:
            // chi is in LDS), count the photons kept, publish, resolve, then
            // update the parents and write the kept photons.
#pragma unroll 1
            for (int e0 = 0; e0 + wave * 64 < total; e0 += kBlock) {
                const int e = e0 + tid;
                const bool valid = e < total;
                const int le = valid ? ev_loc(e) : 0;
                const T cs = valid ? s_chi[le] : T(1);
                const double u0 = dev::draws<sizeof(T) == 4>(a.seed, static_cast<unsigned long long>(S.id_base + c.begin + le),
                                             a.step, static_cast<unsigned long long>(S.species), 0ULL).u[0];
                const float nv = net_sample(valid, cs, u0, e0 / kBlock);
                const bool have = valid && !__builtin_isnan(nv);
                const T xi = valid ? sample_of(have, have ? static_cast<T>(nv) : cs, u0) : T(0);
                if (valid) s_chi[le] = xi;
            }
            __syncthreads();
            for (int e0 = 0; e0 < total; e0 += kBlock) {
                const int e = e0 + tid;
                bool keep = false;
                if (e < total) {
                    const int le = ev_loc(e);
                    const int64_t j = c.begin + le;
                    const double ux = su * ld<T>(S.p[0], j), uy = su * ld<T>(S.p[1], j), uz = su * ld<T>(S.p[2], j);
                    const double u2 = ux * ux + uy * uy + uz * uz;
                    const T gg = static_cast<T>(u2 / (sqrt(1.0 + u2) + 1.0)) * s_chi[le];
                    keep = gg >= static_cast<T>(a.photon_min_energy);
                }
                const unsigned long long m = __ballot(keep);
                if (lane == 0) kmask[(e0 >> 6) + wave] = m;
            }
            __syncthreads();
            if (wave == 0) {
                const int nm = (total + 63) >> 6;
                const int cnt = static_cast<int>(lane) < nm ? __popcll(kmask[lane]) : 0;
                int incl = cnt;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int v = __shfl_up(incl, o);
                    if (static_cast<int>(lane) >= o) incl += v;
                }
                if (static_cast<int>(lane) < kMasks) kpref[lane] = incl - cnt;
                if (lane == 63) {
                    s_kept = incl;
                    publish(a, k, c, static_cast<unsigned long long>(incl));
                }
            }
            __syncthreads();
            prods = s_kept;
            {
                const long long excl = resolve(a, k, c, static_cast<unsigned long long>(prods),
                                               a.stats ? a.stats + QED_STAT_SCAN_TIMEOUT : nullptr, s_lbp, s_lbsum);
                if (tid == 0) s_excl = excl;
            }
            __syncthreads();
            const long long slot0 = s_excl;
#pragma unroll 1
            for (int e = tid; e < total; e += kBlock) {
                const int le = ev_loc(e);
                const int64_t j = c.begin + le;
                const T ux = su * ld<T>(S.p[0], j), uy = su * ld<T>(S.p[1], j), uz = su * ld<T>(S.p[2], j);
                const T w = S.p[10] ? ld<T>(S.p[10], j) : T(1);
                const int64_t parent = S.id_base + j;
                const dev::Draws d = dev::draws<sizeof(T) == 4>(a.seed, static_cast<unsigned long long>(parent), a.step,
                                                static_cast<unsigned long long>(S.species), 0ULL);
                const T xi = s_chi[le];
                const T t1 = dev::neg_log_uniform<T>(d.u[1]);
                const T t2 = dev::neg_log_uniform<T>(d.u[2]);
                const double dx = ux, dy = uy, dz = uz;
                const double u2 = dx * dx + dy * dy + dz * dz;
                const T gg = static_cast<T>(u2 / (sqrt(1.0 + u2) + 1.0)) * xi;
                const T um = static_cast<T>(sqrt(u2));
                const T sc = um > T(0) ? gg / um : T(0);
                const T px = sc * ux, py = sc * uy, pz = sc * uz;
                stnt<T>(S.p[0], j, (ux - px) * iu);
                stnt<T>(S.p[1], j, (uy - py) * iu);
                stnt<T>(S.p[2], j, (uz - pz) * iu);
                stnt<T>(S.p[9], j, t1);
                const unsigned long long m = kmask[e >> 6];
                if ((m >> (e & 63)) & 1ULL) {
                    const long long rank = kpref[e >> 6] + __popcll(m & ((1ULL << (e & 63)) - 1ULL));
                    write_product<T>(a.ph, s_base0 + slot0 + rank, px * iu, py * iu, pz * iu, w, t2, parent);
                }
            }
        }

        // ---------------- the stream's counts (its last chunk) and statistics
        if (tid == 0) {
            const long long incl = s_excl + prods;
            if (k == c.stream_last) {
                if (photon) {
                    *a.el.count = s_base0 + incl;
                    *a.po.count = s_base1 + incl;
                } else {
                    *a.ph.count = s_base0 + incl;
                }
            }
            n_updates += c.len;
            if (photon) {
                n_bw_events += total;
            } else {
                n_qs_events += total;
                n_kept += prods;
            }
        }
    }
    if (a.stats) {
        auto add = [&](int slot, unsigned long long v) {
            if (v) atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + slot), v);
        };
        if (tid == 0) {
            add(QED_STAT_UPDATES, n_updates);
            add(QED_STAT_QS_EVENTS, n_qs_events);
            add(QED_STAT_BW_EVENTS, n_bw_events);
            add(QED_STAT_PHOTONS_KEPT, n_kept);
        }
        if (lane == 0) {
            add(QED_STAT_SURR_BATCHES, n_surr_batches);
            add(QED_STAT_SURR_FALLBACK, n_surr_fallbacks);
        }
        add(QED_STAT_NONFINITE, n_nonfinite);
    }
}

// Both kernels get a register budget of three waves per SIMD: the streaming
// phase needs waves in flight more than registers (measured 9% faster in
// FP32 than the compiler's own choice for the table path; for the surrogate
// path with two-particle batches, 1.00 ms against 1.14 ms with a budget of
// two waves on the cone workload).
constexpr int kTableWavesPerEu = 3;
constexpr int kSurrWavesPerEu = 3;

template <typename T, int kChiMode>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kTableWavesPerEu)))
step_kernel(StepArgs a) {
    step_body<T, kChiMode, false>(a);
}

template <typename T, int kChiMode>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kSurrWavesPerEu)))
step_kernel_surr(StepArgs a) {
    step_body<T, kChiMode, true>(a);
}

template <typename T, int kChiMode, bool kSurr>
struct StepKernel {
    static constexpr auto fn = step_kernel<T, kChiMode>;
};
template <typename T, int kChiMode>
struct StepKernel<T, kChiMode, true> {
    static constexpr auto fn = step_kernel_surr<T, kChiMode>;
};

// Elementwise kernels (grid-stride) -----------------------------------------
template <typename T, bool kPhoton>
__global__ void __launch_bounds__(256) chi_kernel(ElemArgs a) {
    const SetDev& S = a.set;
    const T su = static_cast<T>(a.units.u), se = static_cast<T>(a.units.e), sb = static_cast<T>(a.units.b);
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < S.n;
         j += int64_t(gridDim.x) * blockDim.x) {
        const dev::ChiGamma cg = dev::chi_of<T, kPhoton>(a.chi_mode, su * ld<T>(S.p[0], j), su * ld<T>(S.p[1], j),
                                                         su * ld<T>(S.p[2], j), se * ld<T>(S.p[3], j),
                                                         se * ld<T>(S.p[4], j), se * ld<T>(S.p[5], j),
                                                         sb * ld<T>(S.p[6], j), sb * ld<T>(S.p[7], j),
                                                         sb * ld<T>(S.p[8], j));
        st<T>(a.chi_out, j, static_cast<T>(cg.chi));
    }
}

template <typename T>
__global__ void __launch_bounds__(256) init_tau_kernel(ElemArgs a) {
    const SetDev& S = a.set;
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < S.n;
         j += int64_t(gridDim.x) * blockDim.x) {
        const dev::Draws d = dev::draws(a.seed, static_cast<unsigned long long>(S.id_base + j), dev::kInitStep,
                                        static_cast<unsigned long long>(S.species), 0ULL);
        st<T>(S.p[9], j, static_cast<T>(-log(d.u[0])));
    }
}

template <typename T, bool kPhoton>
__global__ void __launch_bounds__(256) evolve_kernel(ElemArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* tab = reinterpret_cast<T*>(lds_raw);
    for (int i = threadIdx.x; i < a.table.n_chi; i += blockDim.x) tab[i] = ln_rate_ptr<T>(a.table)[i];
    __syncthreads();
    const SetDev& S = a.set;
    const T dt = static_cast<T>(a.dt);
    const T su = static_cast<T>(a.units.u), se = static_cast<T>(a.units.e), sb = static_cast<T>(a.units.b);
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < S.n;
         j += int64_t(gridDim.x) * blockDim.x) {
        const dev::ChiGamma cg = dev::chi_of<T, kPhoton>(a.chi_mode, su * ld<T>(S.p[0], j), su * ld<T>(S.p[1], j),
                                                         su * ld<T>(S.p[2], j), se * ld<T>(S.p[3], j),
                                                         se * ld<T>(S.p[4], j), se * ld<T>(S.p[5], j),
                                                         sb * ld<T>(S.p[6], j), sb * ld<T>(S.p[7], j),
                                                         sb * ld<T>(S.p[8], j));
        const T rate = kPhoton ? dev::rate_bw<T>(tab, a.table, static_cast<T>(cg.chi), static_cast<T>(cg.gamma))
                               : dev::rate_qs<T>(tab, a.table, static_cast<T>(cg.chi), static_cast<T>(cg.gamma));
        const T tn = ld<T>(S.p[9], j) - rate * dt;
        st<T>(S.p[9], j, tn);
        if (S.flags) S.flags[j] = static_cast<uint8_t>(tn < T(0));
    }
}

// T: arithmetic and array type; S: table storage (S = Bf16 reads the BF16
// copies with FP32 arithmetic, for precision studies).
template <typename T, typename S>
__global__ void __launch_bounds__(256) table_rate_kernel(TableCallArgs a) {
    const S* lr;
    if constexpr (sizeof(S) == 2) lr = reinterpret_cast<const S*>(a.table.ln_rate16);
    else lr = ln_rate_ptr<S>(a.table);
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < a.n; j += int64_t(gridDim.x) * blockDim.x) {
        const T chi = ld<T>(a.a, j), g = ld<T>(a.b, j);
        st<T>(a.out, j, a.process == QED_PROC_BW ? dev::rate_bw<T, S>(lr, a.table, chi, g)
                                                 : dev::rate_qs<T, S>(lr, a.table, chi, g));
    }
}

template <typename T, typename S>
__global__ void __launch_bounds__(256) table_sample_kernel(TableCallArgs a) {
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < a.n; j += int64_t(gridDim.x) * blockDim.x) {
        const T chi = ld<T>(a.a, j), r = ld<T>(a.b, j);
        if (a.process == QED_PROC_BW) {
            bool e;
            st<T>(a.out, j, dev::sample_bw<T, S>(a.table, chi, r, e));
            if (a.sel) a.sel[j] = static_cast<uint8_t>(e);
        } else {
            st<T>(a.out, j, dev::sample_qs_lnxi<T, S>(a.table, chi, r));
        }
    }
}

size_t step_lds_bytes(const StepArgs& a, size_t elem) {
    const int nbw = a.bw.n_chi > 0 ? a.bw.n_chi : 0;
    const int nqs = a.qs.n_chi > 0 ? a.qs.n_chi : 0;
    const bool surr = elem == 4 && (a.use_bw_surr || a.use_qs_surr);
    return elem * (((nbw + 1) & ~1) + ((nqs + 1) & ~1)) + sizeof(uint16_t) * kChunk + elem * kChunk +
           (surr ? kSurrLdsBytes + 16 : 0);
}

template <typename T, bool kSurr>
hipError_t launch_step_t(const StepArgs& a, int grid, hipStream_t s) {
    const size_t lds = step_lds_bytes(a, sizeof(T));
    if (a.chi_mode == QED_CHI_COMP32)
        hipLaunchKernelGGL((StepKernel<T, QED_CHI_COMP32, kSurr>::fn), dim3(grid), dim3(kBlock), lds, s, a);
    else if (a.chi_mode == QED_CHI_FP32)
        hipLaunchKernelGGL((StepKernel<T, QED_CHI_FP32, kSurr>::fn), dim3(grid), dim3(kBlock), lds, s, a);
    else
        hipLaunchKernelGGL((StepKernel<T, QED_CHI_FP64, kSurr>::fn), dim3(grid), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

int elem_grid(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return static_cast<int>(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

size_t step_lds_bytes_for(const StepArgs& a, int dtype) { return step_lds_bytes(a, dtype == QED_FP64 ? 8 : 4); }

hipError_t launch_step(const StepArgs& a, int dtype, int grid, hipStream_t s) {
    if (dtype == QED_FP64) return launch_step_t<double, false>(a, grid, s);
    if (a.use_bw_surr || a.use_qs_surr) return launch_step_t<float, true>(a, grid, s);
    return launch_step_t<float, false>(a, grid, s);
}

namespace {
template <typename T, bool kSurr>
int occupancy(const StepArgs& a, size_t lds) {
    int per_cu = 0;
    hipError_t e;
    if (a.chi_mode == QED_CHI_COMP32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, StepKernel<T, QED_CHI_COMP32, kSurr>::fn, kBlock, lds);
    else if (a.chi_mode == QED_CHI_FP32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, StepKernel<T, QED_CHI_FP32, kSurr>::fn, kBlock, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, StepKernel<T, QED_CHI_FP64, kSurr>::fn, kBlock, lds);
    return (e == hipSuccess && per_cu > 0) ? per_cu : 1;
}
}  // namespace

// Persistent grid: as many blocks as fit on the device at once (never more
// than there are chunks), for the kernel variant and LDS size of this launch.
int step_grid_size(const StepArgs& a, int dtype, int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    const bool surr = a.use_bw_surr || a.use_qs_surr;
    int per_cu;
    if (dtype == QED_FP64) per_cu = occupancy<double, false>(a, step_lds_bytes(a, 8));
    else if (surr) per_cu = occupancy<float, true>(a, step_lds_bytes(a, 4));
    else per_cu = occupancy<float, false>(a, step_lds_bytes(a, 4));
    return cus * per_cu;
}

hipError_t launch_table_rate(const TableCallArgs& a, int dtype, hipStream_t s) {
    const int g = elem_grid(a.n);
    if (dtype == QED_FP64) hipLaunchKernelGGL((table_rate_kernel<double, double>), dim3(g), dim3(256), 0, s, a);
    else if (dtype == QED_BF16) hipLaunchKernelGGL((table_rate_kernel<float, dev::Bf16>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((table_rate_kernel<float, float>), dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_table_sample(const TableCallArgs& a, int dtype, hipStream_t s) {
    const int g = elem_grid(a.n);
    if (dtype == QED_FP64) hipLaunchKernelGGL((table_sample_kernel<double, double>), dim3(g), dim3(256), 0, s, a);
    else if (dtype == QED_BF16) hipLaunchKernelGGL((table_sample_kernel<float, dev::Bf16>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((table_sample_kernel<float, float>), dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_chi(const ElemArgs& a, int dtype, hipStream_t s) {
    const int g = elem_grid(a.set.n);
    if (dtype == QED_FP64) {
        if (a.is_photon) hipLaunchKernelGGL((chi_kernel<double, true>), dim3(g), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((chi_kernel<double, false>), dim3(g), dim3(256), 0, s, a);
    } else {
        if (a.is_photon) hipLaunchKernelGGL((chi_kernel<float, true>), dim3(g), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((chi_kernel<float, false>), dim3(g), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_init_tau(const ElemArgs& a, int dtype, hipStream_t s) {
    const int g = elem_grid(a.set.n);
    if (dtype == QED_FP64) hipLaunchKernelGGL((init_tau_kernel<double>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((init_tau_kernel<float>), dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_evolve(const ElemArgs& a, int dtype, hipStream_t s) {
    const int g = std::min(elem_grid(a.set.n), 2048);
    const size_t lds = (dtype == QED_FP64 ? 8 : 4) * static_cast<size_t>(a.table.n_chi);
    if (dtype == QED_FP64) {
        if (a.is_photon) hipLaunchKernelGGL((evolve_kernel<double, true>), dim3(g), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((evolve_kernel<double, false>), dim3(g), dim3(256), lds, s, a);
    } else {
        if (a.is_photon) hipLaunchKernelGGL((evolve_kernel<float, true>), dim3(g), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((evolve_kernel<float, false>), dim3(g), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace qedmi
