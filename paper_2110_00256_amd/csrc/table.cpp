// Table objects: generation, host<->file, upload to the device in FP64,
// FP32 and BF16 (paper Sec. 3.3: tables computed in double precision can be
// stored in single precision; Sec. 5: tables may be stored on disk and
// loaded when needed).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"
#include "tablegen.hpp"

using namespace qedmi;

namespace {

bool check_params(const qed_table_params* p) {
    if (!p) { set_error("params is null"); return false; }
    if (p->process != QED_PROC_BW && p->process != QED_PROC_QS) { set_error("unknown process"); return false; }
    if (p->n_chi < 2 || p->n_chi > 4096) { set_error("n_chi must be in [2, 4096]"); return false; }
    if (p->n_frac < 3 || p->n_frac > 4096) { set_error("n_frac must be in [3, 4096]"); return false; }
    if (!(p->chi_min > 0.0) || !(p->chi_max > p->chi_min) || !std::isfinite(p->chi_max)) {
        set_error("need 0 < chi_min < chi_max < inf");
        return false;
    }
    if (p->process == QED_PROC_QS && !(p->frac_min > 0.0 && p->frac_min < 1.0)) {
        set_error("QS frac_min must be in (0, 1)");
        return false;
    }
    return true;
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ULL) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ULL;
    }
    return h;
}

uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;          // NaN
    const uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);        // nearest even
    return static_cast<uint16_t>((u + rounding) >> 16);
}

void free_device(qed_table* t) {
    if (t->device < 0) return;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(t->device);
    hipFree(t->d_ln_rate64);
    hipFree(t->d_cdf64);
    hipFree(t->d_ln_rate32);
    hipFree(t->d_cdf32);
    hipFree(t->d_cdf16);
    hipFree(t->d_ln_rate16);
    hipSetDevice(cur);
    t->d_ln_rate64 = nullptr;
    t->d_cdf64 = nullptr;
    t->d_ln_rate32 = nullptr;
    t->d_cdf32 = nullptr;
    t->d_cdf16 = nullptr;
    t->d_ln_rate16 = nullptr;
    t->device = -1;
}

const char kMagic[8] = {'Q', 'E', 'D', 'M', 'I', 'T', 'B', '1'};

}  // namespace

qedmi::TableDev qed_table::view() const {
    TableDev v{};
    v.ln_rate64 = d_ln_rate64;
    v.cdf64 = d_cdf64;
    v.ln_rate32 = d_ln_rate32;
    v.cdf32 = d_cdf32;
    v.cdf16 = d_cdf16;
    v.ln_rate16 = d_ln_rate16;
    v.n_chi = p.n_chi;
    v.n_frac = p.n_frac;
    v.chi_min = p.chi_min;
    v.chi_max = p.chi_max;
    v.ln_chi_min = std::log(p.chi_min);
    v.inv_dlnchi = (p.n_chi - 1) / (std::log(p.chi_max) - std::log(p.chi_min));
    v.frac_min = p.frac_min;
    v.ln_frac_min = p.process == QED_PROC_QS ? std::log(p.frac_min) : 0.0;
    v.inv_chi_min = 1.0 / p.chi_min;
    v.ln_chi_max = std::log(p.chi_max);
    v.chi_min_f = static_cast<float>(v.chi_min);
    v.chi_max_f = static_cast<float>(v.chi_max);
    v.ln_chi_min_f = static_cast<float>(v.ln_chi_min);
    v.inv_dlnchi_f = static_cast<float>(v.inv_dlnchi);
    v.ln_frac_min_f = static_cast<float>(v.ln_frac_min);
    v.inv_chi_min_f = static_cast<float>(v.inv_chi_min);
    v.ln_chi_max_f = static_cast<float>(v.ln_chi_max);
    return v;
}

extern "C" int32_t qed_table_generate(const qed_table_params* params, qed_table** out) {
    if (!out) { set_error("out is null"); return QED_ERR_INVALID; }
    *out = nullptr;
    if (!check_params(params)) return QED_ERR_INVALID;
    qed_table* t = new (std::nothrow) qed_table;
    if (!t) { set_error("host allocation failed"); return QED_ERR_ALLOC; }
    t->p = *params;
    try {
        t->ln_rate.assign(params->n_chi, 0.0);
        t->cdf.assign(static_cast<size_t>(params->n_chi) * params->n_frac, 0.0);
    } catch (...) {
        delete t;
        set_error("host allocation failed");
        return QED_ERR_ALLOC;
    }
    generate_tables(params->process, params->chi_min, params->chi_max, params->n_chi, params->n_frac,
                    params->frac_min, params->n_threads, t->ln_rate.data(), t->cdf.data());
    *out = t;
    return QED_OK;
}

extern "C" int32_t qed_table_generate_device(const qed_table_params* params, qed_table** out, void* stream) {
    if (!out) { set_error("out is null"); return QED_ERR_INVALID; }
    *out = nullptr;
    if (!check_params(params)) return QED_ERR_INVALID;
    qed_table* t = new (std::nothrow) qed_table;
    if (!t) { set_error("host allocation failed"); return QED_ERR_ALLOC; }
    t->p = *params;
    try {
        t->ln_rate.assign(params->n_chi, 0.0);
        t->cdf.assign(static_cast<size_t>(params->n_chi) * params->n_frac, 0.0);
    } catch (...) {
        delete t;
        set_error("host allocation failed");
        return QED_ERR_ALLOC;
    }
    const int32_t r = generate_tables_device(*params, t->ln_rate.data(), t->cdf.data(),
                                             static_cast<hipStream_t>(stream));
    if (r) {
        delete t;
        return r;
    }
    *out = t;
    return QED_OK;
}

extern "C" int32_t qed_table_from_host(const qed_table_params* params, const double* ln_rate, const double* cdf,
                                       qed_table** out) {
    if (!out) { set_error("out is null"); return QED_ERR_INVALID; }
    *out = nullptr;
    if (!check_params(params)) return QED_ERR_INVALID;
    if (!ln_rate || !cdf) { set_error("ln_rate/cdf is null"); return QED_ERR_INVALID; }
    qed_table* t = new (std::nothrow) qed_table;
    if (!t) { set_error("host allocation failed"); return QED_ERR_ALLOC; }
    t->p = *params;
    t->ln_rate.assign(ln_rate, ln_rate + params->n_chi);
    t->cdf.assign(cdf, cdf + static_cast<size_t>(params->n_chi) * params->n_frac);
    *out = t;
    return QED_OK;
}

extern "C" int32_t qed_table_save(const qed_table* t, const char* path) {
    if (!t || !path) { set_error("table/path is null"); return QED_ERR_INVALID; }
    FILE* f = std::fopen(path, "wb");
    if (!f) { set_error(std::string("cannot open ") + path); return QED_ERR_IO; }
    const size_t nc = t->cdf.size();
    uint64_t h = fnv1a(&t->p, sizeof(t->p));
    h = fnv1a(t->ln_rate.data(), sizeof(double) * t->ln_rate.size(), h);
    h = fnv1a(t->cdf.data(), sizeof(double) * nc, h);
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&t->p, sizeof(t->p), 1, f) == 1 &&
              std::fwrite(t->ln_rate.data(), sizeof(double), t->ln_rate.size(), f) == t->ln_rate.size() &&
              std::fwrite(t->cdf.data(), sizeof(double), nc, f) == nc && std::fwrite(&h, 8, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) { set_error(std::string("write failed: ") + path); return QED_ERR_IO; }
    return QED_OK;
}

extern "C" int32_t qed_table_load(const char* path, qed_table** out) {
    if (!path || !out) { set_error("path/out is null"); return QED_ERR_INVALID; }
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) { set_error(std::string("cannot open ") + path); return QED_ERR_IO; }
    char magic[8];
    qed_table_params p{};
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, kMagic, 8) != 0 ||
        std::fread(&p, sizeof(p), 1, f) != 1) {
        std::fclose(f);
        set_error("not a table file");
        return QED_ERR_IO;
    }
    if (!check_params(&p)) {
        std::fclose(f);
        set_error("corrupt table header");
        return QED_ERR_IO;
    }
    qed_table* t = new (std::nothrow) qed_table;
    if (!t) { std::fclose(f); set_error("host allocation failed"); return QED_ERR_ALLOC; }
    t->p = p;
    t->ln_rate.resize(p.n_chi);
    t->cdf.resize(static_cast<size_t>(p.n_chi) * p.n_frac);
    uint64_t stored = 0;
    const bool ok = std::fread(t->ln_rate.data(), sizeof(double), p.n_chi, f) == size_t(p.n_chi) &&
                    std::fread(t->cdf.data(), sizeof(double), t->cdf.size(), f) == t->cdf.size() &&
                    std::fread(&stored, 8, 1, f) == 1;
    std::fclose(f);
    uint64_t h = fnv1a(&t->p, sizeof(t->p));
    h = fnv1a(t->ln_rate.data(), sizeof(double) * t->ln_rate.size(), h);
    h = fnv1a(t->cdf.data(), sizeof(double) * t->cdf.size(), h);
    if (!ok || h != stored) {
        delete t;
        set_error("table file short or checksum mismatch");
        return QED_ERR_IO;
    }
    *out = t;
    return QED_OK;
}

extern "C" int32_t qed_table_host_data(const qed_table* t, const double** ln_rate, const double** cdf,
                                       qed_table_params* params) {
    if (!t) { set_error("table is null"); return QED_ERR_INVALID; }
    if (ln_rate) *ln_rate = t->ln_rate.data();
    if (cdf) *cdf = t->cdf.data();
    if (params) *params = t->p;
    return QED_OK;
}

extern "C" int32_t qed_table_to_device(qed_table* t, void* stream) {
    if (!t) { set_error("table is null"); return QED_ERR_INVALID; }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { set_error("hipGetDevice failed"); return QED_ERR_HIP; }
    free_device(t);
    const size_t nr = t->ln_rate.size();
    // CDF rows on the device in row-pair order: entry (n, k) holds
    // (P[n][k], P[n+1][k]) side by side, n < n_chi - 1, so that the sampling
    // search reads both rows it interpolates between with one load
    const size_t nf = static_cast<size_t>(t->p.n_frac), npair = static_cast<size_t>(t->p.n_chi - 1);
    const size_t nc = 2 * npair * nf;
    std::vector<double> c64(nc);
    for (size_t n = 0; n < npair; ++n)
        for (size_t k = 0; k < nf; ++k) {
            c64[2 * (n * nf + k)] = t->cdf[n * nf + k];
            c64[2 * (n * nf + k) + 1] = t->cdf[(n + 1) * nf + k];
        }
    std::vector<float> r32(nr), c32(nc);
    std::vector<uint16_t> c16(nc), r16(nr);
    for (size_t i = 0; i < nr; ++i) {
        r32[i] = static_cast<float>(t->ln_rate[i]);
        r16[i] = to_bf16(r32[i]);
    }
    for (size_t i = 0; i < nc; ++i) {
        c32[i] = static_cast<float>(c64[i]);
        c16[i] = to_bf16(c32[i]);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMalloc(&t->d_ln_rate64, nr * 8) != hipSuccess || hipMalloc(&t->d_cdf64, nc * 8) != hipSuccess ||
        hipMalloc(&t->d_ln_rate32, nr * 4) != hipSuccess || hipMalloc(&t->d_cdf32, nc * 4) != hipSuccess ||
        hipMalloc(&t->d_cdf16, nc * 2) != hipSuccess || hipMalloc(&t->d_ln_rate16, nr * 2) != hipSuccess) {
        t->device = dev;
        free_device(t);
        set_error("device allocation failed");
        return QED_ERR_ALLOC;
    }
    t->device = dev;
    // pageable sources: hipMemcpyAsync stages them before returning
    if (hipMemcpyAsync(t->d_ln_rate64, t->ln_rate.data(), nr * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_cdf64, c64.data(), nc * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_ln_rate32, r32.data(), nr * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_cdf32, c32.data(), nc * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_cdf16, c16.data(), nc * 2, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_ln_rate16, r16.data(), nr * 2, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("table upload failed");
        return QED_ERR_HIP;
    }
    return QED_OK;
}

extern "C" void qed_table_destroy(qed_table* t) {
    if (!t) return;
    free_device(t);
    delete t;
}
