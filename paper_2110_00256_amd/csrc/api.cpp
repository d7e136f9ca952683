// C-ABI layer: argument validation, contexts, chunk tables, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "constants.hpp"
#include "internal.hpp"
#include "surrogate_api.hpp"

using namespace qedmi;

namespace qedmi {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace qedmi

namespace {

int32_t hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return QED_ERR_HIP;
}

bool is_lepton(int sp) { return sp == QED_ELECTRON || sp == QED_POSITRON; }

int32_t check_particles(const qed_particles* p, bool need_fields) {
    if (!p) { set_error("particles is null"); return QED_ERR_INVALID; }
    if (p->n < 0) { set_error("particles.n < 0"); return QED_ERR_INVALID; }
    if (p->dtype != QED_FP64 && p->dtype != QED_FP32) { set_error("particles.dtype must be FP64 or FP32"); return QED_ERR_INVALID; }
    if (p->species < QED_ELECTRON || p->species > QED_ION) { set_error("unknown species"); return QED_ERR_INVALID; }
    if (p->id_base < 0) { set_error("id_base < 0"); return QED_ERR_INVALID; }
    if (p->n == 0 || p->species == QED_ION) return QED_OK;
    if (need_fields) {
        const void* req[10] = {p->ux, p->uy, p->uz, p->ex, p->ey, p->ez, p->bx, p->by, p->bz, p->tau};
        for (const void* q : req)
            if (!q) { set_error("a particle array pointer is null"); return QED_ERR_INVALID; }
    }
    return QED_OK;
}

int32_t check_append(const qed_append* a, int dtype, const char* name) {
    if (!a) { set_error(std::string(name) + " append buffer is null"); return QED_ERR_INVALID; }
    if (!a->count) { set_error(std::string(name) + ".count is null"); return QED_ERR_INVALID; }
    if (a->capacity < 0) { set_error(std::string(name) + ".capacity < 0"); return QED_ERR_INVALID; }
    if (a->dtype != dtype) { set_error(std::string(name) + ".dtype differs from the particles'"); return QED_ERR_INVALID; }
    if (a->capacity > 0 && (!a->ux || !a->uy || !a->uz || !a->w || !a->tau)) {
        set_error(std::string(name) + " has a null array");
        return QED_ERR_INVALID;
    }
    return QED_OK;
}

int32_t check_table(const qed_table* t, int process, const char* name) {
    if (!t) { set_error(std::string(name) + " table is null"); return QED_ERR_INVALID; }
    if (t->p.process != process) { set_error(std::string(name) + " table has the wrong process"); return QED_ERR_INVALID; }
    if (t->device < 0 || !t->d_ln_rate64) { set_error(std::string(name) + " table is not on the device"); return QED_ERR_STATE; }
    if (t->p.n_chi > kMaxTableChi) { set_error("runtime tables are limited to 1024 chi points"); return QED_ERR_INVALID; }
    return QED_OK;
}

SetDev to_set(const qed_particles& p, uint8_t* flags) {
    SetDev s{};
    void* arr[11] = {p.ux, p.uy, p.uz, p.ex, p.ey, p.ez, p.bx, p.by, p.bz, p.tau, p.w};
    for (int i = 0; i < 11; ++i) s.p[i] = arr[i];
    s.n = p.n;
    s.id_base = p.id_base;
    s.species = p.species;
    s.stream = is_lepton(p.species) ? 0 : (p.species == QED_PHOTON ? 1 : -1);
    s.flags = flags;
    return s;
}

AppendDev to_append(const qed_append* a) {
    AppendDev d{};
    if (!a) return d;
    d.ux = a->ux;
    d.uy = a->uy;
    d.uz = a->uz;
    d.w = a->w;
    d.tau = a->tau;
    d.parent = a->parent;
    d.count = a->count;
    d.capacity = a->capacity;
    return d;
}

// Grow the context's device scratch to hold n_chunks chunks (look-back
// status words, chunk table) and n_tiles tiles (tile list, builder order and
// start arrays).  Growth waits for queued work before freeing the old
// buffers; a steady workload never grows.
int32_t reserve(qed_context* ctx, int64_t n_chunks, int64_t n_tiles) {
    n_chunks = std::max<int64_t>(n_chunks, 1);
    n_tiles = std::max<int64_t>(n_tiles, 1);
    if (n_chunks > ctx->status_cap || n_chunks > ctx->chunks_cap) {
        const int64_t cap = std::max<int64_t>(n_chunks, 2 * ctx->status_cap);
        unsigned long long* st = nullptr;
        ChunkDesc* ch = nullptr;
        if (hipMalloc(&st, sizeof(unsigned long long) * cap) != hipSuccess ||
            hipMalloc(&ch, sizeof(ChunkDesc) * cap) != hipSuccess) {
            hipFree(st);
            set_error("device allocation of scan scratch failed");
            return QED_ERR_ALLOC;
        }
        if (hipMemset(st, 0, sizeof(unsigned long long) * cap) != hipSuccess) {
            hipFree(st);
            hipFree(ch);
            set_error("memset of scan scratch failed");
            return QED_ERR_HIP;
        }
        // old scratch may still be in use by queued work: wait before freeing
        hipDeviceSynchronize();
        hipFree(ctx->d_status);
        hipFree(ctx->d_chunks);
        ctx->d_status = st;
        ctx->d_chunks = ch;
        ctx->status_cap = cap;
        ctx->chunks_cap = cap;
        ctx->layout_valid = false;
    }
    if (n_tiles > ctx->tiles_cap) {
        const int64_t cap = std::max<int64_t>(n_tiles, 2 * ctx->tiles_cap);
        int64_t* t = nullptr;
        int32_t* q = nullptr;
        if (hipMalloc(&t, sizeof(int64_t) * 3 * cap) != hipSuccess ||
            hipMalloc(&q, sizeof(int32_t) * 2 * cap) != hipSuccess) {
            hipFree(t);
            set_error("device allocation of the tile list failed");
            return QED_ERR_ALLOC;
        }
        hipDeviceSynchronize();
        hipFree(ctx->d_tiles);
        hipFree(ctx->d_part);
        ctx->d_tiles = t;
        ctx->d_part = q;
        ctx->tiles_cap = cap;
        ctx->layout_valid = false;
    }
    return QED_OK;
}

// Copy the caller's tile list to the device through pinned staging, with no
// host synchronisation: the copy reads buffer `stage_next`, which is reused
// only after the copy issued from it two calls earlier has completed.
int32_t stage_tiles(qed_context* ctx, const int64_t* tiles, int32_t n_tiles, hipStream_t s) {
    const int64_t words = 3 * static_cast<int64_t>(n_tiles);
    if (words > ctx->stage_cap) {
        const int64_t cap = std::max<int64_t>(words, 2 * ctx->stage_cap);
        for (int i = 0; i < 2; ++i) {
            if (ctx->stage_ev[i]) hipEventSynchronize(ctx->stage_ev[i]);
            hipHostFree(ctx->h_stage[i]);
            ctx->h_stage[i] = nullptr;
        }
        ctx->stage_cap = 0;
        for (int i = 0; i < 2; ++i) {
            if (hipHostMalloc(reinterpret_cast<void**>(&ctx->h_stage[i]), sizeof(int64_t) * cap) != hipSuccess) {
                set_error("pinned host allocation of the tile staging failed");
                return QED_ERR_ALLOC;
            }
            if (!ctx->stage_ev[i] && hipEventCreateWithFlags(&ctx->stage_ev[i], hipEventDisableTiming) != hipSuccess) {
                set_error("event creation failed");
                return QED_ERR_HIP;
            }
        }
        ctx->stage_cap = cap;
    }
    const int i = ctx->stage_next;
    ctx->stage_next ^= 1;
    hipError_t e = hipEventSynchronize(ctx->stage_ev[i]);   // the copy of two calls ago
    if (e != hipSuccess) return hip_fail(e, "tile staging wait");
    std::memcpy(ctx->h_stage[i], tiles, sizeof(int64_t) * words);
    e = hipMemcpyAsync(ctx->d_tiles, ctx->h_stage[i], sizeof(int64_t) * words, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(ctx->stage_ev[i], s);
    return e == hipSuccess ? QED_OK : hip_fail(e, "tile list upload");
}

}  // namespace

namespace qedmi {
int32_t check_append_dtype(const qed_append* a, int dtype, const char* name) { return check_append(a, dtype, name); }
AppendDev append_view(const qed_append* a) { return to_append(a); }

// Grow the context's general scratch to at least `bytes` (contents undefined).
int32_t reserve_scratch(qed_context* ctx, int64_t bytes) {
    if (bytes <= ctx->scratch_cap) return QED_OK;
    const int64_t cap = std::max<int64_t>(bytes, 2 * ctx->scratch_cap);
    void* p = nullptr;
    if (hipMalloc(&p, static_cast<size_t>(cap)) != hipSuccess) {
        set_error("device allocation of scratch failed");
        return QED_ERR_ALLOC;
    }
    hipDeviceSynchronize();   // queued work may still use the old buffer
    hipFree(ctx->d_scratch);
    ctx->d_scratch = p;
    ctx->scratch_cap = cap;
    return QED_OK;
}
}  // namespace qedmi

namespace {

// Persistent grid of the step kernel variant this launch uses, queried
// once per variant and LDS size.
int cached_grid(qed_context* ctx, const StepArgs& a, int dtype) {
    const int surr = (a.use_bw_surr || a.use_qs_surr) ? 1 : 0;
    const size_t lds = step_lds_bytes_for(a, dtype);
    for (const auto& g : ctx->grids)
        if (g.dtype == dtype && g.surr == surr && g.chi_mode == a.chi_mode && g.lds == lds) return g.grid;
    const int grid = step_grid_size(a, dtype, ctx->device);
    ctx->grids.push_back({dtype, surr, a.chi_mode, lds, grid});
    return grid;
}

}  // namespace

extern "C" const char* qed_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* qed_version(void) { return "qedmi 0.1 (gfx950)"; }

extern "C" int32_t qed_context_create(int32_t device, qed_context** out) {
    if (!out) { set_error("out is null"); return QED_ERR_INVALID; }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return hip_fail(e == hipSuccess ? hipErrorNoDevice : e, "no HIP device");
    if (device < 0 || device >= n) { set_error("device index out of range"); return QED_ERR_INVALID; }
    qed_context* c = new (std::nothrow) qed_context;
    if (!c) { set_error("host allocation failed"); return QED_ERR_ALLOC; }
    c->device = device;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(device);
    hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, device);
    e = hipMalloc(&c->d_ticket, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c->d_ticket, 0, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    hipSetDevice(cur);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "context allocation");
    }
    *out = c;
    return QED_OK;
}

extern "C" int32_t qed_context_set_units(qed_context* ctx, const qed_units* units) {
    if (!ctx || !units) { set_error("context/units is null"); return QED_ERR_INVALID; }
    Units u;
    constexpr double kPi = 3.141592653589793;
    switch (units->system) {
        case QED_UNITS_SI:
            break;
        case QED_UNITS_NORM_OMEGA:
        case QED_UNITS_NORM_LAMBDA: {
            if (!(units->ref > 0.0) || !std::isfinite(units->ref)) { set_error("reference must be > 0"); return QED_ERR_INVALID; }
            // c = e = m_e = 1 with reference angular frequency w (or w = 2 pi c / lambda)
            const double w = units->system == QED_UNITS_NORM_OMEGA ? units->ref : 2.0 * kPi * kC / units->ref;
            u.e = kMe * kC * w / kQe;
            u.b = kMe * w / kQe;
            u.t = 1.0 / w;
            u.length = kC / w;
            break;
        }
        case QED_UNITS_HL_MEV: {
            // hbar = c = eps0 = 1, energy unit 1 MeV; the HL charge is sqrt(4 pi alpha)
            const double mev = 1e6 * kQe;                          // J
            const double me_mev = kMe * kC * kC / mev;
            const double e_hl = std::sqrt(4.0 * kPi * kAlpha);
            u.e = e_hl * mev * mev / (kHbar * kC * kQe);           // V/m per MeV^2
            u.b = u.e / kC;                                         // T per MeV^2
            u.u = 1.0 / me_mev;                                     // p in MeV/c -> p/(m_e c)
            u.inv_u = me_mev;
            u.t = kHbar / mev;                                      // s per MeV^-1
            u.length = kHbar * kC / mev;                            // m per MeV^-1
            u.energy = 1.0 / me_mev;
            break;
        }
        default:
            set_error("unknown unit system");
            return QED_ERR_INVALID;
    }
    u.e_f = static_cast<float>(u.e);
    u.b_f = static_cast<float>(u.b);
    u.u_f = static_cast<float>(u.u);
    u.inv_u_f = static_cast<float>(u.inv_u);
    ctx->units = u;
    return QED_OK;
}

extern "C" void qed_context_destroy(qed_context* c) {
    if (!c) return;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    hipFree(c->d_ticket);
    hipFree(c->d_status);
    hipFree(c->d_chunks);
    hipFree(c->d_tiles);
    hipFree(c->d_part);
    hipFree(c->d_scratch);
    for (int i = 0; i < 2; ++i) {
        hipHostFree(c->h_stage[i]);
        if (c->stage_ev[i]) hipEventDestroy(c->stage_ev[i]);
    }
    hipSetDevice(cur);
    delete c;
}

static int32_t chi_common(qed_context* ctx, const qed_particles* p, int32_t chi_mode, void* chi_out, void* stream,
                          bool photon) {
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    int32_t r = check_particles(p, true);
    if (r) return r;
    if (photon != (p->species == QED_PHOTON) || p->species == QED_ION) {
        set_error(photon ? "qed_chi_photon needs photons" : "qed_chi_lepton needs electrons or positrons");
        return QED_ERR_INVALID;
    }
    if (chi_mode < QED_CHI_FP64 || chi_mode > QED_CHI_FP32) { set_error("bad chi_mode"); return QED_ERR_INVALID; }
    if (p->n == 0) return QED_OK;
    if (!chi_out) { set_error("chi_out is null"); return QED_ERR_INVALID; }
    ElemArgs a{};
    a.set = to_set(*p, nullptr);
    a.units = ctx->units;
    a.chi_out = chi_out;
    a.chi_mode = chi_mode;
    a.is_photon = photon;
    const hipError_t e = launch_chi(a, p->dtype, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QED_OK : hip_fail(e, "chi launch");
}

extern "C" int32_t qed_chi_lepton(qed_context* ctx, const qed_particles* p, int32_t chi_mode, void* chi_out,
                                  void* stream) {
    return chi_common(ctx, p, chi_mode, chi_out, stream, false);
}
extern "C" int32_t qed_chi_photon(qed_context* ctx, const qed_particles* p, int32_t chi_mode, void* chi_out,
                                  void* stream) {
    return chi_common(ctx, p, chi_mode, chi_out, stream, true);
}

extern "C" int32_t qed_init_optical_depth(qed_context* ctx, qed_particles* p, uint64_t seed, void* stream) {
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    if (!p) { set_error("particles is null"); return QED_ERR_INVALID; }
    int32_t r = check_particles(p, false);
    if (r) return r;
    if (p->n == 0 || p->species == QED_ION) return QED_OK;
    if (!p->tau) { set_error("tau is null"); return QED_ERR_INVALID; }
    ElemArgs a{};
    a.set = to_set(*p, nullptr);
    a.seed = seed;
    const hipError_t e = launch_init_tau(a, p->dtype, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QED_OK : hip_fail(e, "init launch");
}

extern "C" int32_t qed_evolve_optical_depth(qed_context* ctx, const qed_table* rate, qed_particles* p, double dt,
                                            int32_t chi_mode, uint8_t* flags, void* stream) {
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    int32_t r = check_particles(p, true);
    if (r) return r;
    if (p->species == QED_ION) { set_error("ions carry no optical depth"); return QED_ERR_INVALID; }
    const bool photon = p->species == QED_PHOTON;
    r = check_table(rate, photon ? QED_PROC_BW : QED_PROC_QS, photon ? "BW" : "QS");
    if (r) return r;
    if (!std::isfinite(dt) || dt < 0.0) { set_error("dt must be finite and >= 0"); return QED_ERR_INVALID; }
    if (chi_mode < QED_CHI_FP64 || chi_mode > QED_CHI_FP32) { set_error("bad chi_mode"); return QED_ERR_INVALID; }
    if (p->n == 0) return QED_OK;
    ElemArgs a{};
    a.set = to_set(*p, flags);
    a.table = rate->view();
    a.dt = dt * ctx->units.t;
    a.units = ctx->units;
    a.chi_mode = chi_mode;
    a.is_photon = photon;
    const hipError_t e = launch_evolve(a, p->dtype, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QED_OK : hip_fail(e, "evolve launch");
}

namespace qedmi {

int32_t prepare_sets(const qed_step_desc* d, bool generate_only, StepArgs& a, int& dtype) {
    if (!d) { set_error("desc is null"); return QED_ERR_INVALID; }
    if (d->n_sets <= 0 || d->n_sets > kMaxSets || !d->sets) { set_error("need 1..8 particle sets"); return QED_ERR_INVALID; }
    if (d->n_tiles < 0 || (d->n_tiles > 0 && !d->tiles)) { set_error("bad tiles"); return QED_ERR_INVALID; }
    if (!generate_only && (!std::isfinite(d->dt) || d->dt < 0.0)) { set_error("dt must be finite and >= 0"); return QED_ERR_INVALID; }
    if (!(d->photon_min_energy >= 0.0)) { set_error("photon_min_energy must be >= 0"); return QED_ERR_INVALID; }
    if (!(d->chi_qed_min >= 0.0)) { set_error("chi_qed_min must be >= 0"); return QED_ERR_INVALID; }
    if (d->chi_mode < QED_CHI_FP64 || d->chi_mode > QED_CHI_FP32) { set_error("bad chi_mode"); return QED_ERR_INVALID; }
    a = StepArgs{};
    dtype = d->sets[0].dtype;
    for (int i = 0; i < d->n_sets; ++i) {
        const qed_particles& p = d->sets[i];
        int32_t r = check_particles(&p, true);
        if (r) return r;
        if (p.dtype != dtype) { set_error("all sets must share one dtype"); return QED_ERR_INVALID; }
        uint8_t* fl = d->flags ? d->flags[i] : nullptr;
        if (generate_only && !fl && p.n > 0 && p.species != QED_ION) { set_error("flags required"); return QED_ERR_INVALID; }
        a.sets[i] = to_set(p, fl);
    }
    a.n_sets = d->n_sets;
    a.generate_only = generate_only ? 1 : 0;
    return QED_OK;
}

int32_t prepare_tables(const Units& units, const qed_step_desc* d, StepArgs& a, int dtype) {
    bool any_lepton = false, any_photon = false;
    for (int i = 0; i < a.n_sets; ++i) {
        if (a.sets[i].n > 0 && a.sets[i].stream == 0) any_lepton = true;
        if (a.sets[i].n > 0 && a.sets[i].stream == 1) any_photon = true;
    }
    if (any_photon) {
        int32_t r = check_table(d->bw, QED_PROC_BW, "BW");
        if (!r) r = check_append(d->electrons, dtype, "electrons");
        if (!r) r = check_append(d->positrons, dtype, "positrons");
        if (r) return r;
        a.bw = d->bw->view();
    }
    if (any_lepton) {
        int32_t r = check_table(d->qs, QED_PROC_QS, "QS");
        if (!r) r = check_append(d->photons, dtype, "photons");
        if (r) return r;
        a.qs = d->qs->view();
    }
    a.ph = to_append(any_lepton ? d->photons : nullptr);
    a.el = to_append(any_photon ? d->electrons : nullptr);
    a.po = to_append(any_photon ? d->positrons : nullptr);
    a.stats = d->stats;
    a.dt = d->dt * units.t;
    a.dt_f = static_cast<float>(a.dt);
    a.units = units;
    a.seed = d->seed;
    a.step = d->step;
    a.photon_min_energy = d->photon_min_energy * units.energy;
    a.chi_qed_min = d->chi_qed_min;
    a.drag = (2.0 / 3.0) * kRateR0 * a.dt;
    a.chi_mode = dtype == QED_FP64 ? QED_CHI_FP64 : d->chi_mode;
    if ((d->bw_surrogate || d->qs_surrogate) && dtype != QED_FP32) {
        set_error("surrogate sampling runs on the FP32 path only");
        return QED_ERR_INVALID;
    }
    return surrogate_bind(a, d->bw_surrogate, d->qs_surrogate);
}

int32_t plan_chunks(const StepArgs& a, const int64_t* tiles, int32_t n_tiles, int32_t* idx, ChunkPlan& plan) {
    plan = ChunkPlan{};
    const int nt = tiles ? n_tiles : a.n_sets;
    int64_t per_stream[2] = {0, 0};
    int64_t chunks[2] = {0, 0};
    int32_t parts[2] = {0, 0};
    int64_t last_end[kMaxSets];
    for (int i = 0; i < kMaxSets; ++i) last_end[i] = 0;
    bool ordered = true;   // every set's (non-empty) tiles come in increasing, disjoint order
    for (int t = 0; t < nt; ++t) {
        const int64_t set = tiles ? tiles[3 * t] : t;
        const int64_t b = tiles ? tiles[3 * t + 1] : 0;
        const int64_t e = tiles ? tiles[3 * t + 2] : a.sets[t].n;
        if (set < 0 || set >= a.n_sets || b < 0 || e < b || e > a.sets[set].n) {
            set_error("tile out of range of its set");
            return QED_ERR_INVALID;
        }
        if (e == b) continue;
        if (b < last_end[set]) ordered = false;
        last_end[set] = std::max(last_end[set], e);
        const int stream = a.sets[set].stream;
        if (stream < 0) continue;   // ions: passed through, never read
        per_stream[stream] += e - b;
        chunks[stream] += (e - b + kChunk - 1) / kChunk;
        parts[stream] += 1;
    }
    if (!ordered) {
        // sort the non-empty tiles by (set, begin) and look for an overlap
        int m = 0;
        for (int t = 0; t < nt; ++t)
            if (tiles[3 * t + 2] > tiles[3 * t + 1]) idx[m++] = t;
        std::sort(idx, idx + m, [tiles](int32_t x, int32_t y) {
            return tiles[3 * x] != tiles[3 * y] ? tiles[3 * x] < tiles[3 * y] : tiles[3 * x + 1] < tiles[3 * y + 1];
        });
        for (int i = 1; i < m; ++i) {
            const int32_t p = idx[i - 1], q = idx[i];
            if (tiles[3 * p] == tiles[3 * q] && tiles[3 * q + 1] < tiles[3 * p + 2]) {
                set_error("tiles of one set overlap");
                return QED_ERR_INVALID;
            }
        }
    }
    if (per_stream[0] >= (1LL << kStatusBits) || per_stream[1] >= (1LL << kStatusBits)) {
        set_error("more than 2^30 - 1 particles in one product stream");
        return QED_ERR_INVALID;
    }
    if (chunks[0] + chunks[1] > INT_MAX / 2) { set_error("too many chunks"); return QED_ERR_INVALID; }
    plan.n_tiles = nt;
    plan.n_part0 = parts[0];
    plan.n_part = parts[0] + parts[1];
    plan.n_chunks0 = static_cast<int32_t>(chunks[0]);
    plan.n_chunks = static_cast<int32_t>(chunks[0] + chunks[1]);
    return QED_OK;
}

ChunkBuildArgs chunk_build_args(const StepArgs& a, const ChunkPlan& plan) {
    ChunkBuildArgs b{};
    b.n_tiles = plan.n_tiles;
    b.n_part0 = plan.n_part0;
    b.n_part = plan.n_part;
    b.n_chunks0 = plan.n_chunks0;
    b.n_chunks = plan.n_chunks;
    for (int i = 0; i < a.n_sets; ++i) {
        b.set_stream[i] = a.sets[i].stream;
        b.set_n[i] = a.sets[i].n;
    }
    return b;
}

}  // namespace qedmi

static int32_t run_chunks(qed_context* ctx, const qed_step_desc* d, bool generate_only, hipStream_t s) {
    // the descriptor and its tiles are checked first (no HIP call), then
    // the context, the tables and the buffers
    StepArgs a;
    int dtype = 0;
    int32_t r = prepare_sets(d, generate_only, a, dtype);
    if (r) return r;
    const int64_t* tiles = d->n_tiles > 0 ? d->tiles : nullptr;
    std::vector<int32_t> local_idx;
    std::vector<int32_t>& idx = ctx ? ctx->tile_idx : local_idx;
    if (tiles && idx.size() < static_cast<size_t>(d->n_tiles)) idx.resize(d->n_tiles);
    ChunkPlan plan;
    r = plan_chunks(a, tiles, d->n_tiles, idx.data(), plan);
    if (r) return r;
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    int dev = 0;
    hipGetDevice(&dev);
    if (dev != ctx->device) { set_error("context belongs to another device"); return QED_ERR_INVALID; }
    r = prepare_tables(ctx->units, d, a, dtype);
    if (r) return r;
    if (plan.n_chunks == 0) return QED_OK;
    r = reserve(ctx, plan.n_chunks, plan.n_tiles);
    if (r) return r;
    // the chunk table on the device is rebuilt only when the layout (set
    // sizes and streams, tile list) differs from the one it was built for
    std::vector<int64_t>& key = ctx->layout_key;
    const size_t klen = 2 + 2 * static_cast<size_t>(a.n_sets) + (tiles ? 3 * static_cast<size_t>(d->n_tiles) : 0);
    bool same = ctx->layout_valid && key.size() == klen && key[0] == a.n_sets && key[1] == (tiles ? d->n_tiles : -1);
    for (int i = 0; same && i < a.n_sets; ++i)
        same = key[2 + 2 * i] == a.sets[i].n && key[3 + 2 * i] == a.sets[i].stream;
    if (same && tiles)
        same = std::memcmp(key.data() + 2 + 2 * a.n_sets, tiles, sizeof(int64_t) * 3 * d->n_tiles) == 0;
    if (!same) {
        ctx->layout_valid = false;
        if (tiles) {
            r = stage_tiles(ctx, tiles, d->n_tiles, s);
            if (r) return r;
        }
        ChunkBuildArgs b = chunk_build_args(a, plan);
        b.tiles = tiles ? ctx->d_tiles : nullptr;
        b.order = ctx->d_part;
        b.ostart = ctx->d_part + ctx->tiles_cap;
        b.chunks = ctx->d_chunks;
        const hipError_t e = launch_chunk_build(b, s);
        if (e != hipSuccess) return hip_fail(e, "chunk table build");
        key.assign(klen, 0);
        key[0] = a.n_sets;
        key[1] = tiles ? d->n_tiles : -1;
        for (int i = 0; i < a.n_sets; ++i) {
            key[2 + 2 * i] = a.sets[i].n;
            key[3 + 2 * i] = a.sets[i].stream;
        }
        if (tiles) std::memcpy(key.data() + 2 + 2 * a.n_sets, tiles, sizeof(int64_t) * 3 * d->n_tiles);
        ctx->layout_valid = true;
    }
    a.n_chunks = plan.n_chunks;
    const int grid = std::max(1, std::min(a.n_chunks, cached_grid(ctx, a, dtype)));
    ctx->epoch = ctx->epoch + 1 == 0 ? 1 : ctx->epoch + 1;
    a.status = ctx->d_status;
    a.ticket = ctx->d_ticket;
    a.ticket_base = ctx->ticket_issued;
    a.epoch = ctx->epoch;
    a.chunks = ctx->d_chunks;
    const hipError_t e = launch_step(a, dtype, grid, s);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    // every block takes exactly one failing ticket before it exits
    ctx->ticket_issued += static_cast<unsigned long long>(a.n_chunks) + static_cast<unsigned long long>(grid);
    return QED_OK;
}

extern "C" int32_t qed_step(qed_context* ctx, const qed_step_desc* d, void* stream) {
    return run_chunks(ctx, d, false, static_cast<hipStream_t>(stream));
}

extern "C" int32_t qed_generate_pairs(qed_context* ctx, const qed_table* bw, qed_particles* photons,
                                      const uint8_t* flags, uint64_t seed, uint64_t step, int32_t chi_mode,
                                      qed_append* electrons, qed_append* positrons, void* stream) {
    if (!photons) { set_error("photons is null"); return QED_ERR_INVALID; }
    if (photons->species != QED_PHOTON) { set_error("qed_generate_pairs needs photons"); return QED_ERR_INVALID; }
    if (!flags && photons->n > 0) { set_error("flags is null"); return QED_ERR_INVALID; }
    qed_step_desc d{};
    uint8_t* fl[1] = {const_cast<uint8_t*>(flags)};
    d.bw = bw;
    d.sets = photons;
    d.n_sets = 1;
    d.electrons = electrons;
    d.positrons = positrons;
    d.flags = fl;
    d.seed = seed;
    d.step = step;
    d.chi_mode = chi_mode;
    return run_chunks(ctx, &d, true, static_cast<hipStream_t>(stream));
}

extern "C" int32_t qed_generate_photon_and_update_momentum(qed_context* ctx, const qed_table* qs,
                                                           qed_particles* leptons, const uint8_t* flags,
                                                           uint64_t seed, uint64_t step, int32_t chi_mode,
                                                           double photon_min_energy, qed_append* photons,
                                                           void* stream) {
    if (!leptons) { set_error("leptons is null"); return QED_ERR_INVALID; }
    if (!is_lepton(leptons->species)) { set_error("photon emission needs electrons or positrons"); return QED_ERR_INVALID; }
    if (!flags && leptons->n > 0) { set_error("flags is null"); return QED_ERR_INVALID; }
    qed_step_desc d{};
    uint8_t* fl[1] = {const_cast<uint8_t*>(flags)};
    d.qs = qs;
    d.sets = leptons;
    d.n_sets = 1;
    d.photons = photons;
    d.flags = fl;
    d.seed = seed;
    d.step = step;
    d.chi_mode = chi_mode;
    d.photon_min_energy = photon_min_energy;
    return run_chunks(ctx, &d, true, static_cast<hipStream_t>(stream));
}

static int32_t table_call(const qed_table* t, int32_t dtype, const void* a, const void* b, void* out, uint8_t* sel,
                          int64_t n, void* stream, bool sample) {
    if (!t) { set_error("table is null"); return QED_ERR_INVALID; }
    if (t->device < 0 || !t->d_ln_rate64) { set_error("table is not on the device"); return QED_ERR_STATE; }
    if (dtype != QED_FP64 && dtype != QED_FP32 && dtype != QED_BF16) {
        set_error("dtype must be FP64, FP32 or BF16");
        return QED_ERR_INVALID;
    }
    if (n < 0) { set_error("n < 0"); return QED_ERR_INVALID; }
    if (n == 0) return QED_OK;
    if (!a || !b || !out) { set_error("null array"); return QED_ERR_INVALID; }
    TableCallArgs c{};
    c.table = t->view();
    c.a = a;
    c.b = b;
    c.out = out;
    c.sel = sel;
    c.n = n;
    c.process = t->p.process;
    const hipError_t e = sample ? launch_table_sample(c, dtype, static_cast<hipStream_t>(stream))
                                : launch_table_rate(c, dtype, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QED_OK : hip_fail(e, "table kernel launch");
}

extern "C" int32_t qed_table_rate(const qed_table* t, int32_t dtype, const void* chi, const void* gamma,
                                  void* rate_out, int64_t n, void* stream) {
    return table_call(t, dtype, chi, gamma, rate_out, nullptr, n, stream, false);
}

extern "C" int32_t qed_table_sample(const qed_table* t, int32_t dtype, const void* chi, const void* u, void* out,
                                    uint8_t* electron_selected, int64_t n, void* stream) {
    return table_call(t, dtype, chi, u, out, electron_selected, n, stream, true);
}

extern "C" int32_t qed_read_count(const qed_append* a, int64_t* host_count, void* stream) {
    if (!a || !a->count || !host_count) { set_error("append/count/host_count is null"); return QED_ERR_INVALID; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(host_count, a->count, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "count readback");
    if (*host_count > a->capacity) {
        set_error("products exceeded the append buffer capacity");
        return QED_ERR_CAPACITY;
    }
    return QED_OK;
}
