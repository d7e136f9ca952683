// C-ABI layer: argument validation, contexts, chunk tables, launches.
#include <hip/hip_runtime.h>

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

// Ensure the context's scratch can hold n chunks.
int32_t reserve(qed_context* ctx, int64_t n_chunks) {
    if (n_chunks <= ctx->status_cap && n_chunks <= ctx->chunks_cap) return QED_OK;
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
    ctx->h_chunks_cached.clear();
    return QED_OK;
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

// Build chunks ordered by (stream, tile order) and upload them if they
// differ from the cached table.
int32_t build_chunks(qed_context* ctx, const std::vector<SetDev>& sets, const int64_t* tiles, int n_tiles,
                     hipStream_t s, int32_t* n_chunks_out) {
    std::vector<int64_t> tl;
    if (tiles) {
        tl.assign(tiles, tiles + 3 * static_cast<size_t>(n_tiles));
    } else {
        for (size_t i = 0; i < sets.size(); ++i) {
            tl.push_back(static_cast<int64_t>(i));
            tl.push_back(0);
            tl.push_back(sets[i].n);
        }
        n_tiles = static_cast<int>(sets.size());
    }
    std::vector<ChunkDesc> ch;
    int64_t per_stream[2] = {0, 0};
    for (int stream = 0; stream < 2; ++stream) {
        const int first = static_cast<int>(ch.size());
        for (int t = 0; t < n_tiles; ++t) {
            const int64_t set = tl[3 * t], b = tl[3 * t + 1], e = tl[3 * t + 2];
            if (set < 0 || set >= static_cast<int64_t>(sets.size()) || b < 0 || e < b || e > sets[set].n) {
                set_error("tile out of range of its set");
                return QED_ERR_INVALID;
            }
            if (sets[set].stream != stream) continue;
            per_stream[stream] += e - b;
            for (int64_t x = b; x < e; x += kChunk) {
                ChunkDesc c{};
                c.begin = x;
                c.set = static_cast<int32_t>(set);
                c.len = static_cast<int32_t>(std::min<int64_t>(kChunk, e - x));
                c.stream = stream;
                c.stream_first = first;
                ch.push_back(c);
            }
        }
        for (size_t i = first; i < ch.size(); ++i) ch[i].stream_last = static_cast<int32_t>(ch.size() - 1);
    }
    if (per_stream[0] >= (1LL << kStatusBits) || per_stream[1] >= (1LL << kStatusBits)) {
        set_error("more than 2^30 - 1 particles in one product stream");
        return QED_ERR_INVALID;
    }
    if (ch.size() > static_cast<size_t>(INT_MAX / 2)) { set_error("too many chunks"); return QED_ERR_INVALID; }
    const int32_t r = reserve(ctx, std::max<int64_t>(1, static_cast<int64_t>(ch.size())));
    if (r != QED_OK) return r;
    const bool same = ch.size() == ctx->h_chunks_cached.size() &&
                      (ch.empty() || std::memcmp(ch.data(), ctx->h_chunks_cached.data(),
                                                 ch.size() * sizeof(ChunkDesc)) == 0);
    if (!same && !ch.empty()) {
        ctx->h_chunks_cached = ch;   // kept alive: the async copy reads it
        const hipError_t e = hipMemcpyAsync(ctx->d_chunks, ctx->h_chunks_cached.data(), ch.size() * sizeof(ChunkDesc),
                                            hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "chunk table upload");
        hipStreamSynchronize(s);
    }
    *n_chunks_out = static_cast<int32_t>(ch.size());
    return QED_OK;
}

int32_t launch_chunks(qed_context* ctx, StepArgs& a, int dtype, hipStream_t s) {
    if (a.n_chunks == 0) return QED_OK;
    int dev = 0;
    hipGetDevice(&dev);
    if (dev != ctx->device) { set_error("context belongs to another device"); return QED_ERR_INVALID; }
    const int grid = std::max(1, std::min(a.n_chunks, step_grid_size(a, dtype, ctx->device)));
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
    hipFree(c->d_scratch);
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

static int32_t run_chunks(qed_context* ctx, const qed_step_desc* d, bool generate_only, hipStream_t s) {
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    if (!d) { set_error("desc is null"); return QED_ERR_INVALID; }
    if (d->n_sets <= 0 || d->n_sets > kMaxSets || !d->sets) { set_error("need 1..8 particle sets"); return QED_ERR_INVALID; }
    if (d->n_tiles < 0 || (d->n_tiles > 0 && !d->tiles)) { set_error("bad tiles"); return QED_ERR_INVALID; }
    if (!generate_only && (!std::isfinite(d->dt) || d->dt < 0.0)) { set_error("dt must be finite and >= 0"); return QED_ERR_INVALID; }
    if (!(d->photon_min_energy >= 0.0)) { set_error("photon_min_energy must be >= 0"); return QED_ERR_INVALID; }
    if (!(d->chi_qed_min >= 0.0)) { set_error("chi_qed_min must be >= 0"); return QED_ERR_INVALID; }
    if (d->chi_mode < QED_CHI_FP64 || d->chi_mode > QED_CHI_FP32) { set_error("bad chi_mode"); return QED_ERR_INVALID; }
    const int dtype = d->sets[0].dtype;
    bool any_lepton = false, any_photon = false;
    std::vector<SetDev> sets;
    for (int i = 0; i < d->n_sets; ++i) {
        const qed_particles& p = d->sets[i];
        int32_t r = check_particles(&p, true);
        if (r) return r;
        if (p.dtype != dtype) { set_error("all sets must share one dtype"); return QED_ERR_INVALID; }
        uint8_t* fl = d->flags ? d->flags[i] : nullptr;
        if (generate_only && !fl && p.n > 0 && p.species != QED_ION) { set_error("flags required"); return QED_ERR_INVALID; }
        if (p.n > 0 && is_lepton(p.species)) any_lepton = true;
        if (p.n > 0 && p.species == QED_PHOTON) any_photon = true;
        sets.push_back(to_set(p, fl));
    }
    StepArgs a{};
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
    int32_t n_chunks = 0;
    int32_t r = build_chunks(ctx, sets, d->n_tiles > 0 ? d->tiles : nullptr, d->n_tiles, s, &n_chunks);
    if (r) return r;
    for (size_t i = 0; i < sets.size(); ++i) a.sets[i] = sets[i];
    a.n_sets = static_cast<int32_t>(sets.size());
    a.n_chunks = n_chunks;
    a.generate_only = generate_only ? 1 : 0;
    a.ph = to_append(any_lepton ? d->photons : nullptr);
    a.el = to_append(any_photon ? d->electrons : nullptr);
    a.po = to_append(any_photon ? d->positrons : nullptr);
    a.stats = d->stats;
    a.dt = d->dt * ctx->units.t;
    a.units = ctx->units;
    a.seed = d->seed;
    a.step = d->step;
    a.photon_min_energy = d->photon_min_energy * ctx->units.energy;
    a.chi_qed_min = d->chi_qed_min;
    a.drag = (2.0 / 3.0) * kRateR0 * a.dt;
    a.chi_mode = dtype == QED_FP64 ? QED_CHI_FP64 : d->chi_mode;
    if ((d->bw_surrogate || d->qs_surrogate) && dtype != QED_FP32) {
        set_error("surrogate sampling runs on the FP32 path only");
        return QED_ERR_INVALID;
    }
    r = surrogate_bind(a, d->bw_surrogate, d->qs_surrogate);
    if (r) return r;
    return launch_chunks(ctx, a, dtype, s);
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
