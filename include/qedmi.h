/*
 * qedmi.h -- C ABI of the MI355X strong-field QED Monte Carlo library.
 *
 * The library implements the per-timestep QED sub-step that a particle-in-
 * cell code adds to its loop (Fedeli et al., "PICSAR-QED", arXiv:2110.00256,
 * Fig. 1 and Sec. 3): the quantum parameter chi of each macro-particle, the
 * optical-depth evolution with the tabulated total rates of nonlinear
 * Breit-Wheeler pair production (BW) and quantum-synchrotron photon emission
 * (QS), and, on an event, inverse-CDF sampling of the product, creation of
 * the photon or pair, parent recoil and optical-depth redraw.
 *
 * Conventions shared by every call:
 *   Units      momentum u = p/(m_e c) (dimensionless); E in V/m; B in T;
 *              dt in s.  Photons carry u with gamma_gamma = |u|.
 *   Memory     particle arrays and product buffers are caller-owned DEVICE
 *              memory (SoA, one array per component, element type given by
 *              `dtype`).  Tables, contexts and surrogates are library-owned
 *              opaque handles.  Host pointers are marked "host".
 *   Streams    `stream` is a hipStream_t passed as void* (NULL = default
 *              stream).  Every device call is asynchronous on that stream;
 *              only the calls documented as synchronous block the host.
 *   Contexts   a qed_context owns per-device scratch (look-back status words,
 *              chunk tickets, chunk tables).  Calls that share a context must
 *              be ordered on one stream; concurrent calls on one context race.
 *   Errors     every call returns int32_t: QED_OK (0) or a negative
 *              qed_status; qed_last_error() gives a thread-local message.
 *              Nothing aborts and no exception crosses the ABI.  Argument
 *              checks happen on the host before any launch; a call that
 *              returns an error has launched nothing.
 *   Randomness every uniform comes from Philox4x64-10 (Salmon et al., SC'11)
 *              with key (seed, 0) and counter (particle id, step, species,
 *              block); the id of element i is id_base + i.  Results are
 *              therefore independent of launch shape and bit-reproducible.
 *              The paper leaves the generator to the caller (Sec. 3.3); this
 *              library fixes a counter-based one so that results can be
 *              reproduced exactly on the CPU.
 */
#ifndef QEDMI_H
#define QEDMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QED_OK = 0,
    QED_ERR_INVALID = -1,   /* bad argument (null pointer, size, enum, range) */
    QED_ERR_HIP = -2,       /* a HIP runtime call failed                      */
    QED_ERR_ALLOC = -3,     /* host or device allocation failed               */
    QED_ERR_CAPACITY = -4,  /* product buffer too small (see qed_read_count)  */
    QED_ERR_IO = -5,        /* file missing, short or corrupt                 */
    QED_ERR_STATE = -6      /* object not ready (e.g. table not on device)    */
} qed_status;

typedef enum { QED_FP64 = 0, QED_FP32 = 1, QED_BF16 = 2 } qed_dtype;
typedef enum { QED_PROC_BW = 0, QED_PROC_QS = 1 } qed_process;
typedef enum { QED_ELECTRON = 0, QED_POSITRON = 1, QED_PHOTON = 2, QED_ION = 3 } qed_species;

/* How chi is evaluated on FP32 particle data (FP64 data always uses FP64).
 * QED_CHI_FP64: FP64 arithmetic on the FP32 inputs (default).
 * QED_CHI_COMP32: FP32 pair ("double-float") arithmetic with error-free
 *   transformations (TwoSum, TwoProd via fma) throughout.
 * QED_CHI_FP32: plain FP32 (for precision studies only). */
typedef enum { QED_CHI_FP64 = 0, QED_CHI_COMP32 = 1, QED_CHI_FP32 = 2 } qed_chi_mode;

/* ------------------------------------------------------------------ tables
 * Lookup tables of Sec. 3.1 (BW) and Sec. 3.2 (QS).  Grid: n_chi points
 * ln chi_n = ln chi_min + n (ln chi_max - ln chi_min)/(n_chi - 1).
 *   BW: ln_rate[n] = ln T(chi_n); cdf[n][m] = P(chi_n, xi_m), xi_m =
 *       0.5 m/(n_frac - 1) (only xi <= 1/2 is stored, by the symmetry
 *       P(xi) = 1 - P(1 - xi)).
 *   QS: ln_rate[n] = ln G(chi_n); cdf[n][m] = ln P(chi_n, xi_m), ln xi_m =
 *       ln frac_min (1 - m/(n_frac - 1)).
 * cdf is row-major [n_chi][n_frac]. */
typedef struct {
    int32_t process;     /* qed_process                                   */
    int32_t n_chi;       /* >= 2, <= 4096                                 */
    int32_t n_frac;      /* >= 3, <= 4096                                 */
    int32_t n_threads;   /* host threads for generation; <= 0: all cores  */
    double chi_min;      /* > 0                                           */
    double chi_max;      /* > chi_min                                     */
    double frac_min;     /* QS xi_min in (0, 1); ignored for BW           */
} qed_table_params;

typedef struct qed_table qed_table;

/* Generate both tables of one process from the Bessel-function integrals of
 * Sec. 2.1 (T(chi_gamma), BW differential rate) or Sec. 2.2 (G(chi), S(chi,
 * xi)), in FP64 on the host (the paper's generation is CPU-side, Sec. 3).
 * Synchronous.  *out receives a new handle (caller destroys it). */
int32_t qed_table_generate(const qed_table_params* params, qed_table** out);

/* The same tables generated on the current device: every entry is an FP64
 * quadrature in HIP (one thread per table interval, composite Gauss-Legendre
 * in each interval's natural variable, Bessel functions from their integral
 * representation).  The paper generates tables on the CPU only (Sec. 3);
 * results agree with qed_table_generate to about 1e-10.  Synchronous on
 * `stream`; the FP64 host master copy is filled as for qed_table_generate
 * (call qed_table_to_device to upload the runtime copies). */
int32_t qed_table_generate_device(const qed_table_params* params, qed_table** out, void* stream);

/* Wrap caller-provided FP64 host arrays (copied) as a table (e.g. tables
 * produced elsewhere, Sec. 5: "load a lookup table generated beforehand"). */
int32_t qed_table_from_host(const qed_table_params* params, const double* ln_rate,
                            const double* cdf, qed_table** out);

/* Save / load: little-endian header, parameters, FP64 payload, FNV-1a
 * checksum.  load returns QED_ERR_IO on a missing, short or corrupt file. */
int32_t qed_table_save(const qed_table* t, const char* path);
int32_t qed_table_load(const char* path, qed_table** out);

/* Borrow the FP64 host arrays (valid until destroy) and the parameters. */
int32_t qed_table_host_data(const qed_table* t, const double** ln_rate, const double** cdf,
                            qed_table_params* params);

/* Copy the table to the current device in FP64, FP32 and BF16 (BF16 for
 * precision studies).  The device CDF is stored in row-pair order: entry
 * (n, m), n < n_chi - 1, holds cdf[n][m] and cdf[n+1][m] side by side, so
 * that a sampling probe reads both rows it interpolates between with one
 * load ((n_chi - 1) x n_frac pairs).  Returns after the copies are done (the
 * converted copies are staged in host memory owned by the call). */
int32_t qed_table_to_device(qed_table* t, void* stream);

void qed_table_destroy(qed_table* t);

/* ---------------------------------------------------------------- context */
typedef struct qed_context qed_context;

/* Create a context on `device` (allocates ~ 16 MiB of device scratch). */
int32_t qed_context_create(int32_t device, qed_context** out);
void qed_context_destroy(qed_context* ctx);

/* ------------------------------------------------------------------ units
 * The unit system of the caller's arrays and scalars for every call made
 * through a context (Sec. 4: the interface accepts SI units and normalised
 * units with a reference frequency or length; internally the paper works in
 * Heaviside-Lorentz units with 1 MeV as reference energy).  Default SI:
 * E in V/m, B in T, momenta as u = p/(m_e c), time in s, energies in
 * m_e c^2.  Normalised (c = e = m_e = 1): E in m_e c w/e, B in m_e w/e, time
 * in 1/w, u as in SI, energies in m_e c^2, with w the reference angular
 * frequency given directly or as w = 2 pi c / lambda from a reference
 * wavelength (this library's reading of "reference length").
 * Heaviside-Lorentz (hbar = c = eps0 = 1, unit 1 MeV): E and B in MeV^2
 * (charge sqrt(4 pi alpha)), momenta in MeV/c, time in 1/MeV, energies in
 * MeV.  Tables are dimensionless and shared by all systems.  Applies to
 * qed_chi_*, qed_evolve_optical_depth, qed_step and the generate calls
 * (fields, momenta, dt, photon_min_energy; products are written in the
 * same units); qed_push and the Schwinger calls take SI. */
typedef enum {
    QED_UNITS_SI = 0,
    QED_UNITS_NORM_OMEGA = 1,    /* ref = reference angular frequency (1/s) */
    QED_UNITS_NORM_LAMBDA = 2,   /* ref = reference wavelength (m)          */
    QED_UNITS_HL_MEV = 3         /* ref unused                              */
} qed_unit_system;
typedef struct {
    int32_t system;
    int32_t pad_;
    double ref;
} qed_units;
int32_t qed_context_set_units(qed_context* ctx, const qed_units* units);

/* -------------------------------------------------------------- particles
 * One species' SoA arrays in device memory, n elements of `dtype` each.
 * tau is read and written; u is written by photon emission; w (weight,
 * may be NULL meaning 1) is copied to products. */
typedef struct {
    void *ux, *uy, *uz;
    void *ex, *ey, *ez;
    void *bx, *by, *bz;
    void *tau;
    void *w;
    int64_t n;          /* >= 0                                  */
    int64_t id_base;    /* global id of element 0 (Philox key)   */
    int32_t species;    /* qed_species                           */
    int32_t dtype;      /* QED_FP64 or QED_FP32                  */
} qed_particles;

/* Product (append) buffer: products are written at slots [*count,
 * *count + k) in parent order (tile order, then index), and *count is
 * increased by k.  Slots >= capacity are not written but still counted, so
 * after a call *count holds the size that was needed.  count is DEVICE
 * memory (one int64) owned by the caller, who resets it when the products
 * have been consumed.  parent (may be NULL) receives the parent's id. */
typedef struct {
    void *ux, *uy, *uz, *w, *tau;
    int64_t* parent;
    int64_t* count;
    int64_t capacity;
    int32_t dtype;      /* must equal the parents' dtype */
    int32_t pad_;
} qed_append;

/* ------------------------------------------------------------ runtime calls */

/* chi of each lepton (Sec. 2, quantum parameter of an electron or positron)
 * or photon (chi_gamma), written to chi_out (n elements of the particles'
 * dtype).  Evaluated as sqrt(|a|^2 + (gamma^2 - |u|^2) E_par^2)/E_s with
 * a = gamma E_perp + c u x B, which is the printed formula rewritten so that
 * no two O(gamma^2 E^2) terms are subtracted.  chi_mode applies to FP32. */
int32_t qed_chi_lepton(qed_context* ctx, const qed_particles* p, int32_t chi_mode, void* chi_out,
                       void* stream);
int32_t qed_chi_photon(qed_context* ctx, const qed_particles* p, int32_t chi_mode, void* chi_out,
                       void* stream);

/* tau = -ln u with u the first draw of block (id, step = 2^64 - 1,
 * species, 0): optical depth drawn from p(x) = exp(-x) (Sec. 3). */
int32_t qed_init_optical_depth(qed_context* ctx, qed_particles* p, uint64_t seed, void* stream);

/* tau <- tau - (dN/dt) dt with the BW (photons) or QS (leptons) total rate
 * from `rate` (Sec. 2.1 / 2.2 totals, Sec. 3.1 / 3.2 interpolation), and
 * flags[i] = (tau < 0) (may be NULL).  `rate` must match the species. */
int32_t qed_evolve_optical_depth(qed_context* ctx, const qed_table* rate, qed_particles* p, double dt,
                                 int32_t chi_mode, uint8_t* flags, void* stream);

/* Pair creation for every photon with flags[i] != 0 (Sec. 2.1, Sec. 3.1):
 * sample the electron's chi fraction, append the electron to `electrons`
 * and the positron to `positrons` at the same slot, mark the photon dead
 * (tau = +inf).  Products get tau from the block's 2nd and 3rd draws. */
int32_t qed_generate_pairs(qed_context* ctx, const qed_table* bw, qed_particles* photons,
                           const uint8_t* flags, uint64_t seed, uint64_t step, int32_t chi_mode,
                           qed_append* electrons, qed_append* positrons, void* stream);

/* Photon emission for every lepton with flags[i] != 0 (Sec. 2.2, Sec. 3.2):
 * sample xi, emit a photon of energy (gamma - 1) xi along the lepton's
 * momentum, subtract its momentum from the lepton, redraw the lepton's tau.
 * Photons with energy below photon_min_energy (units of m_e c^2; 0 keeps
 * all) are not appended (Sec. 5), the lepton recoils either way. */
int32_t qed_generate_photon_and_update_momentum(qed_context* ctx, const qed_table* qs,
                                                qed_particles* leptons, const uint8_t* flags,
                                                uint64_t seed, uint64_t step, int32_t chi_mode,
                                                double photon_min_energy, qed_append* photons,
                                                void* stream);

/* Total rate dN/dt in 1/s for n (chi, gamma) pairs (device arrays of
 * `dtype`): BW tables give (alpha m c^2/hbar)(chi/gamma) T(chi) (Sec. 2.1),
 * QS tables (2/3)(alpha m c^2/hbar) G(chi)/gamma (Sec. 2.2), with the
 * table interpolation and out-of-table rules of the step. */
int32_t qed_table_rate(const qed_table* t, int32_t dtype, const void* chi, const void* gamma, void* rate_out,
                       int64_t n, void* stream);

/* Inverse-CDF sample for n (chi, u) pairs, u in (0, 1) (Sec. 3.1 / 3.2
 * sampling).  BW: out = xi in [0, 1/2], electron_selected[i] = (u <= 1/2)
 * (may be NULL).  QS: out = ln xi.  Device arrays of `dtype`.
 * For both calls dtype QED_BF16 means FP32 arrays and FP32 arithmetic on the
 * BF16-stored copies of the tables (precision studies). */
int32_t qed_table_sample(const qed_table* t, int32_t dtype, const void* chi, const void* u, void* out,
                         uint8_t* electron_selected, int64_t n, void* stream);

/* ------------------------------------------------------------- fused step
 * One QED sub-step over several species in a single persistent launch:
 * chi, rate, tau update, event test, and for events the draws, sampling,
 * product creation, parent update and ordered append (the four steps above
 * fused, with products appended in parent order through a decoupled
 * look-back scan).  Leptons (electrons, positrons) emit photons into
 * `photons`; photons create pairs into `electrons` / `positrons`; ions are
 * passed through untouched (never read).
 *
 * tiles (host, may be NULL): n_tiles triples (set, begin, end) splitting
 * set `set` of `sets` into [begin, end) ranges; products follow tile order.
 * NULL means one tile per set, in set order.  Tiles of one set must be
 * disjoint (an overlap is refused with QED_ERR_INVALID before anything is
 * launched); tiles over ions are allowed and skipped.  The tile list is
 * copied during the call (through the context's pinned staging), so the
 * caller may reuse it at once; the chunk table is built on the device and
 * rebuilt only when the tile list or the set sizes change.  The call does
 * not block the host, except when the context's scratch must grow (a larger
 * population or more tiles than any earlier call). */
typedef struct qed_surrogate qed_surrogate;

typedef struct {
    const qed_table* bw;           /* needed if any set is a photon set   */
    const qed_table* qs;           /* needed if any set is a lepton set   */
    const qed_surrogate* bw_surrogate;  /* NULL: table inverse CDF        */
    const qed_surrogate* qs_surrogate;  /* NULL: table inverse CDF        */
    qed_particles* sets;           /* host array of n_sets descriptors    */
    int32_t n_sets;
    int32_t n_tiles;
    const int64_t* tiles;          /* host, 3 * n_tiles, or NULL          */
    qed_append* photons;           /* required if any lepton set          */
    qed_append* electrons;         /* required if any photon set          */
    qed_append* positrons;         /* required if any photon set          */
    uint8_t** flags;               /* host array of n_sets device pointers (entries may be NULL), or NULL */
    int64_t* stats;                /* device, QED_STATS_LEN int64 accumulated (may be NULL) */
    double dt;
    uint64_t seed;
    uint64_t step;
    double photon_min_energy;
    int32_t chi_mode;
    int32_t pad_;
    double chi_qed_min;            /* > 0: below this chi a particle keeps its
                                      optical depth; photons do nothing and
                                      leptons lose the classically radiated
                                      energy (2/3)(alpha m c^2/hbar) chi^2 dt
                                      m c^2 along u (Sec. 6, WarpX's minimum
                                      quantum parameter).  0: off */
} qed_step_desc;

/* stats layout (accumulated, device int64): */
enum {
    QED_STAT_UPDATES = 0,        /* particles updated (ions excluded)      */
    QED_STAT_QS_EVENTS = 1,      /* lepton events                          */
    QED_STAT_BW_EVENTS = 2,      /* photon events                          */
    QED_STAT_PHOTONS_KEPT = 3,   /* photons appended (before capacity)     */
    QED_STAT_SURR_BATCHES = 4,   /* event batches sampled by a surrogate   */
    QED_STAT_SURR_FALLBACK = 5,  /* event batches that fell back to tables */
    QED_STAT_NONFINITE = 6,      /* particles whose chi is not finite or whose
                                    updated optical depth is NaN or -inf (bad
                                    momenta or fields); they are stepped as
                                    the arithmetic gives, only counted here.
                                    +inf (a decayed photon) is not counted */
    QED_STAT_SCAN_TIMEOUT = 7,   /* look-back waits abandoned (must stay 0) */
    QED_STATS_LEN = 8
};

int32_t qed_step(qed_context* ctx, const qed_step_desc* desc, void* stream);

/* qed_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same descriptor, kernels and results as qed_step (bit-identical), but
 * every scratch buffer (chunk ticket, look-back status words, chunk table,
 * tile list) lives in one fixed library array per GPU of 2.81 MiB, held
 * until the process ends; nothing is allocated, on the device or the host,
 * and the host is never synchronised.
 *   ctx     may be NULL (SI units, current device); when given, only its
 *           unit system and device are used, never its scratch.
 *   limits  at most 65536 chunks of 4096 particles (2^28 particles over
 *           all sets, counted per tile) and at most 8192 tiles; larger
 *           inputs return QED_ERR_INVALID before anything is launched.
 *   sharing every call on one GPU uses that GPU's array: calls that overlap
 *           on one GPU (different streams or threads) race.  Calls ordered
 *           on one stream are safe; the array needs no clearing between
 *           them (the ticket is monotonic, status words carry a per-call
 *           epoch and the chunk table is rebuilt by every call).
 * Each call re-uploads the tile list through kernel arguments (one small
 * launch per 160 tiles) and rebuilds the chunk table on the device. */
int32_t qed_step_noalloc(const qed_context* ctx, const qed_step_desc* desc, void* stream);

/* Measurement aid (not part of the method): stream n_bytes (a multiple of
 * 8) of device memory with the fused step's streaming access pattern,
 * non-temporal 8-byte loads and stores in a grid-stride loop.  mode 0 reads
 * src (dst must be a valid device pointer, written only if the data hold a
 * NaN), 1 writes dst, 2 copies src to dst; modes 3 and 4 read and write like
 * 0 and 1 with ordinary (temporal) loads and stores.  Used to scale the hardware's
 * fetch and write counters by what they report for a known byte count. */
int32_t qed_traffic_calibrate(const void* src, void* dst, int64_t n_bytes, int32_t mode, void* stream);

/* Synchronise `stream` and read an append buffer's count to the host;
 * returns QED_ERR_CAPACITY if it exceeds the buffer's capacity. */
int32_t qed_read_count(const qed_append* a, int64_t* host_count, void* stream);

/* ---------------------------------------------------------------- surrogate
 * Learned inverse CDF: an MLP 2 -> 64 -> 64 -> 1 with SiLU activations,
 * BF16 weights and FP32 accumulation, mapping (normalised ln chi, g(u)) to
 * the sampled fraction (ln xi for QS; a scaled xi for BW), trained on
 * samples of the table inverse CDF (Sec. 3.1 / 3.2 sampling) by the
 * library's own BF16-MFMA forward/backward kernels and Adam.  Outside its
 * trained chi range, or when a probe against the table exceeds
 * `probe_tol`, sampling falls back to the table: in the fused step one wave
 * batch of 64 events in `probe_every` is probed, and a wave whose probe
 * fails keeps the table for the rest of its chunk. */
typedef struct {
    int32_t process;        /* qed_process of the table it learns         */
    int32_t n_samples;      /* training set size (e.g. 1 << 24)            */
    int32_t batch;          /* minibatch (multiple of 256)                 */
    int32_t steps;          /* optimiser steps                             */
    float lr;               /* Adam learning rate (cosine decay to lr/100) */
    float probe_tol;        /* allowed |delta| of the output per probe     */
    double chi_lo, chi_hi;  /* trained chi range (inside the table range)  */
    uint64_t seed;
    int32_t probe_every;    /* in the fused step, probe one wave batch in
                               this many (1 = every batch; <= 0 means 1)   */
    int32_t tail_permille;  /* training samples (in 1/1000) whose uniform is
                               drawn evenly in the network's second input
                               (logit u for QS, the normal quantile of the
                               folded r for BW) instead of evenly in u: more
                               of the set in the tails, where the fit's
                               largest CDF errors sit.  0: all even in u   */
    float ks_budget;        /* > 0: after training, the trained chi range is
                               split into QED_SURR_BANDS equal bands in
                               ln chi and the network serves a band only if
                               its largest CDF-space error against the table
                               there, max over u of |P_table(network sample)
                               - u| (the KS distance of the two sampled
                               spectra for a monotone map), stays within
                               ks_budget on 8 chi x 4096 u validation points;
                               the table serves the other bands.  0: the
                               network serves the whole trained range      */
    int32_t pad_;
} qed_surrogate_cfg;

/* Train on the device (table must be on the device).  Synchronous at the
 * end (returns after training); *final_loss (host, may be NULL) receives
 * the mean loss of the last 64 steps. */
int32_t qed_surrogate_train(qed_context* ctx, const qed_table* table, const qed_surrogate_cfg* cfg,
                            qed_surrogate** out, float* final_loss, void* stream);
/* Build from host FP32 master weights (layout below) for tests. */
int32_t qed_surrogate_from_host(const qed_table* table, const qed_surrogate_cfg* cfg,
                                const float* params, qed_surrogate** out);
/* Parameter layout (QED_SURR_NPARAM floats): W1[64][2], b1[64],
 * W2[64][64] (row = output unit), b2[64], W3[64], b3. */
enum { QED_SURR_NPARAM = 64 * 2 + 64 + 64 * 64 + 64 + 64 + 1 };
int32_t qed_surrogate_get_params(const qed_surrogate* s, float* host_params);
/* The validation result: band_err (host, QED_SURR_BANDS floats) receives
 * each band's largest CDF-space error (0 if not validated), *served_mask
 * bit b is set when band b is sampled by the network. */
enum { QED_SURR_BANDS = 64 };
int32_t qed_surrogate_bands(const qed_surrogate* s, float* band_err, uint64_t* served_mask);
/* Forward on n device inputs x[n][2] (FP32) -> y[n] (FP32), BF16 MFMA. */
int32_t qed_surrogate_forward(const qed_surrogate* s, const float* x, float* y, int64_t n, void* stream);
/* Loss and gradient of 0.5 mean((y - t)^2) over one minibatch of device
 * inputs x[n][2], targets t[n]; grad (device, QED_SURR_NPARAM floats) and
 * loss (device, 1 float). */
int32_t qed_surrogate_grad(const qed_surrogate* s, const float* x, const float* t, int64_t n,
                           float* grad, float* loss, void* stream);
/* Sample through the surrogate for n events: chi[n], u[n] (device, FP32)
 * -> out[n] (device FP32: ln xi for QS, xi in [0, 1/2] for BW) with table
 * fallback outside the trained range. */
int32_t qed_surrogate_sample(const qed_surrogate* s, const float* chi, const float* u, float* out,
                             int64_t n, void* stream);
void qed_surrogate_destroy(qed_surrogate* s);

/* ---------------------------------------------------------------- Schwinger
 * Pair creation from the vacuum by a strong field (Sec. 2.3).  Works on
 * field values per grid cell rather than on particles. */
typedef struct {
    const void *ex, *ey, *ez;   /* device arrays, V/m, one entry per cell  */
    const void *bx, *by, *bz;   /* device arrays, T                        */
    int64_t n;                  /* number of cells (>= 0)                  */
    int64_t cell_id_base;       /* global id of cell 0: Philox counter and
                                   the products' parent id                 */
    int32_t dtype;              /* QED_FP64 or QED_FP32                    */
    int32_t pad_;
} qed_cells;

/* Pair production rate per unit volume d2N/(dt dV) in m^-3 s^-1 for every
 * cell, from the field invariants F = (E^2 - c^2 B^2)/2 and G = c E.B
 * (Sec. 2.3 rate formula).  rate_out: device FP64 array of n entries
 * (rates near E_s exceed the FP32 range in SI units), also for FP32 fields.
 * Arithmetic in FP64; the invariants are formed on fields scaled
 * by E_s and without subtracting sqrt(F^2 + G^2) from |F|.  A field with no
 * invariant electric part (pure magnetic, crossed |E| = c|B|) gives 0. */
int32_t qed_schwinger_rate(qed_context* ctx, const qed_cells* cells, void* rate_out, void* stream);

/* Macro-pairs created at rest (Sec. 2.3: pairs may be initialised at rest).
 * The paper gives the rate only; the count per cell is this library's
 * choice: Poisson with mean lambda = rate * cell_volume * dt / weight
 * (inversion with the first uniform of counter (cell id, step, 4, 0)), and
 * for lambda > 25 a Gaussian of mean and variance lambda rounded to the
 * nearest integer and clipped at 0.  Pairs are appended to `electrons` and
 * `positrons` in cell order after their current counts (the two members of a
 * pair at the same offset), with u = 0, w = weight, parent = cell id and
 * tau = -ln u from counter (cell id, step, 4, 1 + i/2) (uniforms 2(i%2) and
 * 2(i%2)+1 of pair i).  The counts are incremented on the device; capacity
 * contract as for qed_step (pairs beyond capacity are not written; check
 * with qed_read_count).  Buffers must have dtype = cells->dtype.
 * cell_volume in m^3, dt in s, weight = physical pairs per macro-pair > 0.
 * The context keeps 8 bytes of device scratch per cell of the largest call
 * (each cell's count, computed once and used to place the pairs). */
int32_t qed_schwinger_pairs(qed_context* ctx, const qed_cells* cells, double cell_volume, double dt,
                            double weight, uint64_t seed, uint64_t step, qed_append* electrons,
                            qed_append* positrons, void* stream);

/* ------------------------------------------------------------------- push
 * A particle push in prescribed analytic fields, to close the loop of the
 * QED sub-step without a field solver: the benchmark geometries of Sec. 5.1
 * (electrons in a static magnetic field perpendicular to their motion, and
 * electrons counter-propagating with a circularly polarised plane wave). */
typedef enum { QED_FIELD_UNIFORM = 0, QED_FIELD_CP_WAVE = 1 } qed_field_kind;
typedef struct {
    int32_t kind;         /* qed_field_kind                                  */
    int32_t direction;    /* CP wave: +1 propagates along +x, -1 along -x    */
    double e0[3];         /* UNIFORM: E (V/m)                                */
    double b0[3];         /* UNIFORM: B (T)                                  */
    double amplitude;     /* CP wave: |E| (V/m); E = A (0, cos ph, sin ph),
                             B = (direction x_hat) x E / c,
                             ph = 2 pi (direction x - c t)/wavelength + phase */
    double wavelength;    /* CP wave: m                                      */
    double phase;         /* CP wave: rad                                    */
} qed_field;

/* Advance one species by dt from time t: leptons by the relativistic Boris
 * scheme (u at half steps, charge -e for electrons and +e for positrons,
 * fields at the old position and time t), photons on straight lines at c;
 * positions x, y, z (device, m, same dtype as the particles) are updated,
 * and the fields at the new position and time t + dt are written into the
 * particles' E/B arrays (what qed_step reads next).  Ions are refused. */
int32_t qed_push(qed_context* ctx, const qed_particles* p, void* x, void* y, void* z, const qed_field* field,
                 double t, double dt, void* stream);

/* ------------------------------------------------------------------- misc */
const char* qed_last_error(void);
/* Library version string. */
const char* qed_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QEDMI_H */
