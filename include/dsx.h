/*
 * dsx -- diffuse scattering from atomistic models on one MI355X (gfx950).
 *
 * C-ABI of the hot path of the FFT method of Paddison, "Ultrafast Calculation
 * of Diffuse Scattering from Atomistic Models" (arXiv:1809.07088):
 *
 *   per-sublattice 3D FFTs of occupancy, spin and Taylor displacement-monomial
 *   fields (Sec. III.B-D), recombined at the supercell Bragg points into the
 *   Bragg-subtracted diffuse intensity I = <|F|^2> - |<F>|^2 (Sec. II Eq.
 *   bragg_diffuse_sf; Sec. III Eqs. comp_diffuse_intensity,
 *   disp_diffuse_intensity, mag_intensity), and the Lanczos windowed-sinc
 *   noise filter (Sec. V.B).
 *
 * Conventions used by every call:
 *   - Plain pointers and sizes only.  "Device" pointers are HIP device
 *     allocations on the current device; "host" pointers are ordinary memory.
 *   - Arrays are C order (last index fastest), float32 unless stated.
 *   - Reciprocal-space points are integer supercell Bragg indices G (Eq. G_def):
 *     G = (G1/n1) a* + (G2/n2) b* + (G3/n3) c*; g = G/n is the same point in
 *     reciprocal-lattice units.  All transforms use the +i sign (Eqs. sf, fft).
 *   - Every function returns DSX_OK (0) or a negative status.  Argument and
 *     state errors return synchronously, enqueue nothing and leave the model
 *     unchanged; dsx_last_error() then gives a message for the calling thread.
 *   - A HIP failure inside a call returns DSX_ERR_DEVICE and marks the model
 *     failed: every later call on it returns DSX_ERR_DEVICE.
 *   - Distinct models may be used from different threads concurrently; one
 *     model must not be used by two threads at once.
 */
#ifndef DSX_H
#define DSX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dsx_model_s* dsx_model;   /* opaque, owned by the library */
typedef int32_t dsx_status;

enum {
    DSX_OK = 0,
    DSX_ERR_ARG = -1,          /* invalid argument                              */
    DSX_ERR_STATE = -2,        /* call-order violation (e.g. sites not all set)  */
    DSX_ERR_NOMEM = -3,        /* device or host allocation failed               */
    DSX_ERR_DEVICE = -4,       /* HIP error; the model is now failed             */
    DSX_ERR_UNSUPPORTED = -5,  /* valid but outside what this build implements   */
    DSX_ERR_BUSY = -6          /* resource held: model recorded in a batch, or a
                                  server's request queue is full                 */
};

enum { DSX_NUCLEAR = 0, DSX_MAGNETIC = 1 };
enum { DSX_HOST = 0, DSX_DEVICE = 1 };

/* Largest supported values (DSX_ERR_UNSUPPORTED beyond them). */
#define DSX_MAX_N        256   /* supercell edge n_alpha                         */
#define DSX_MAX_SITES    64    /* species-sites per unit cell                    */
#define DSX_MAX_ORDER    16    /* Taylor order of exp(i G.u); above 8 the C(N+3,3)   */
                               /* fields of one site (n3/2 + 1 complex values     */
                               /* each) must fit the recombination's LDS          */

/*
 * Model description (Sec. II; Sec. III Eq. r_vec).  An atom of site mu at lattice
 * point R sits at R + r_mu + u_{R,mu} (unit-cell coordinates) with occupancy
 * delta_{R,mu}.  Only the pointers' contents are read, during dsx_create_model.
 */
typedef struct {
    double  cell[6];        /* a, b, c [Angstrom]; alpha, beta, gamma [deg] (Sec. II: a* = 2 pi b x c / V) */
    int32_t n[3];           /* supercell n1, n2, n3 (Eq. r_def), each in [1, DSX_MAX_N]                       */
    int32_t n_sites;        /* species-sites (mu, i), in [1, DSX_MAX_SITES]; several may share a position     */
    const double* frac;     /* [n_sites][3] average fractional positions r_mu (Eq. r_vec)                     */
    const int32_t* pos_id;  /* [n_sites] position index used for the normalisation N, or NULL (= identity)   */
    const double* b;        /* [n_sites] scattering length b_mu (nuclear) or moment scale (magnetic)         */
    const double* ff;       /* [n_sites][7] form factor (A,a,B,b,C,c,D):                                      */
                            /*   f(s) = A e^{-a s^2} + B e^{-b s^2} + C e^{-c s^2} + D, s = |Q|/(4 pi);        */
                            /*   magnetic: f_mag of Eq. mag_sf; nuclear: a |Q|-dependent factor multiplying  */
                            /*   b_mu (X-ray f_j(|Q|), Sec. II), which takes the class form of the           */
                            /*   recombination (sites grouped by r_mu3 and f).  NULL => f = 1.               */
    int32_t kind;           /* DSX_NUCLEAR or DSX_MAGNETIC                                                    */
    int32_t has_occ;        /* 0: delta == 1 everywhere (no occupancy array is read)                         */
    int32_t taylor_order;   /* order N of the Taylor expansion of exp(i G.u) (Sec. III.C, Eq.                */
                            /*   disp_expansion), in [0, DSX_MAX_ORDER]; 0 = no displacements.  Nuclear:     */
                            /*   the displacive structure factor (Eq. total_sf_taylor).  Magnetic: the        */
                            /*   moments stay at R + r_mu and the displacements enter only through the        */
                            /*   Debye-Waller factor T_mu(G) of Eq. mag_sf, per Sec. III.A Eq. dw the mean of  */
                            /*   (1 + a) e^{i G.u} over cells and configurations (1 + a = delta / c_mu, c_mu   */
                            /*   the site's mean occupancy), here its order-N expansion; 0 => T = 1           */
    int32_t n_configs;      /* ensemble size M >= 1 (<.> is the mean over configurations)                    */
    double  norm_N;         /* N of I = <|F|^2>/N (Eq. intensity_sf); 0 => n1 n2 n3 x distinct positions      */
} dsx_model_desc;

/*
 * Host-only plan query: fills the sizes the model would use, without touching a
 * GPU.  fields_per_site = number of real fields transformed per site and
 * configuration: (N+1)(N+2)(N+3)/6 Taylor monomials (Sec. III.C: (n+1)(n+2)/2 per
 * order n), minus the constant one when has_occ == 0; 3 spin components for
 * magnetic models (Sec. III.D, Eq. mag_ft).  device_bytes = resident device
 * memory of the model excluding output boxes.
 */
typedef struct {
    int32_t fields_per_site;
    int32_t total_fields;        /* n_configs x n_sites x fields_per_site          */
    int32_t n_classes;           /* site groups sharing r_mu3 (and form factor)     */
    int32_t reserved;
    int64_t spectrum_bytes;      /* complex64 half spectra of all fields            */
    int64_t device_bytes;
} dsx_plan_info;

dsx_status dsx_plan_query(const dsx_model_desc* d, dsx_plan_info* info);

/*
 * Host-only split-site mapping (Sec. III.B, after Eq. comp_ft): when the
 * displacements of a site take only a few values, every displaced position becomes
 * a site of its own and displacive disorder becomes occupational disorder, which the
 * compositional path (taylor_order 0, has_occ 1) then evaluates exactly, with no
 * Taylor truncation.  Site mu with distinct displacements u_1..u_K (in the order
 * first met, scanning configurations, then cells) becomes K sites at r_mu + u_k with
 * b_mu and occupancy delta_{R,mu} [u_{R,mu} = u_k] (two displacements are equal when
 * every component differs by at most tol; the site's position uses the first one).
 *   n[3], n_sites, frac[n_sites][3], b[n_sites], n_configs   as in dsx_model_desc
 *   occ   [n_configs][n_sites][n1][n2][n3] or NULL (delta = 1)
 *   disp  [n_configs][n_sites][n1][n2][n3][3] fractional unit-cell displacements
 *   max_sites  capacity of the outputs (<= DSX_MAX_SITES)
 * Outputs (host memory owned by the caller): *n_split sites, frac_out[max_sites][3],
 * b_out[max_sites], parent_out[max_sites] (the original site; pass it, or the
 * original pos_id of it, as pos_id so that N is unchanged), occ_out
 * [n_configs][max_sites][n1][n2][n3] (the first *n_split site blocks of each
 * configuration are written).  DSX_ERR_UNSUPPORTED when more than max_sites split
 * sites arise; nothing is written then.
 */
dsx_status dsx_split_sites(const int32_t n[3], int32_t n_sites, const double* frac, const double* b,
                           int32_t n_configs, const float* occ, const float* disp, double tol,
                           int32_t max_sites, int32_t* n_split, double* frac_out, double* b_out,
                           int32_t* parent_out, float* occ_out);

/*
 * Create a model on the current HIP device and allocate its device state
 * (inputs, spectra, FP64 sums).  *out receives the handle.  DSX_ERR_NOMEM when
 * the device cannot hold it.
 */
dsx_status dsx_create_model(const dsx_model_desc* d, dsx_model* out);

/*
 * Set the variables of configuration `config` (0 <= config < n_configs).
 *   occ  [n_sites][n1][n2][n3]     delta (read iff has_occ)
 *   disp [n_sites][n1][n2][n3][3]  u in fractional unit-cell coordinates (read iff
 *                                  taylor_order > 0)
 *   spin [n_sites][n1][n2][n3][3]  Cartesian moment M (read iff magnetic)
 * Pointers not read may be NULL.  where = DSX_HOST or DSX_DEVICE for all three.
 * The data are copied before return (the caller may free them at once).
 */
dsx_status dsx_set_sites(dsx_model m, int32_t config, const float* occ, const float* disp,
                         const float* spin, int32_t where);

/*
 * Stream-ordered form of dsx_set_sites for device arrays: the copies are enqueued
 * on hip_stream after all earlier work of the model (on any stream), so a loop of
 * set_sites_async + compute calls never waits on the host.  The caller keeps the
 * source arrays unchanged until the copies have run on hip_stream.  Not for models
 * owned by a server (DSX_ERR_STATE).
 */
dsx_status dsx_set_sites_async(dsx_model m, int32_t config, const float* occ, const float* disp,
                               const float* spin, void* hip_stream);

/*
 * Output box: the integer points G with g0[a] <= G_a < g0[a] + count[a], count >= 1.
 */
dsx_status dsx_set_grid(dsx_model m, const int32_t g0[3], const int32_t count[3]);

/*
 * I(G) on the box, float32 [count0][count1][count2]:
 *   nuclear   I = (1/N) [ (1/M) sum_m |F_m|^2 - [G = 0 mod n] |(1/M) sum_m F_m|^2 ]
 *             with F_m(G) = sum_{mu} b_mu e^{2 pi i g.r_mu} sum_{p+q+r<=N}
 *             (2 pi i)^{p+q+r} g1^p g2^q g3^r / (p! q! r!) X^{pqr}_{m,mu}(k),
 *             k = G mod n, X the +i FFT of delta u1^p u2^q u3^r (Sec. III.C, Eq.
 *             total_sf_taylor, regrouped by monomial; Sec. III.B for N = 0);
 *   magnetic  I = (C/N) [ (1/M) sum |F_perp|^2 - [G = 0 mod n] |(1/M) sum F_perp|^2 ],
 *             F = sum_mu f_mu(|Q|) T_mu(G) b_mu e^{2 pi i g.r_mu} M_{k,mu}, F_perp = F -
 *             Ghat (Ghat . F), C = 0.07265 barn, I(0) = 0 (Sec. III.D, Eq. mag_sf), with
 *             T_mu(G) = sum_{p+q+r<=N} (2 pi i)^{p+q+r} g1^p g2^q g3^r / (p! q! r!)
 *             <u1^p u2^q u3^r>_mu (Eq. dw at order N; <.>_mu the mean over the site's
 *             occupied atoms and the configurations), T = 1 when taylor_order = 0.
 * The points G = 0 (mod n) are evaluated in float64 from float64 lattice sums.
 * out: device pointer (where = DSX_DEVICE; asynchronous on hip_stream, NULL = the
 * null stream) or host pointer (where = DSX_HOST; synchronous).
 * DSX_ERR_STATE unless every configuration's sites and the grid are set.
 */
dsx_status dsx_compute_intensity(dsx_model m, float* out, int32_t where, void* hip_stream);

/*
 * dsx_compute_intensity for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving or refinement loops, harnesses that forbid it.
 * Same result and output rules as dsx_compute_intensity with where = DSX_DEVICE
 * (out: device pointer; asynchronous on hip_stream, NULL = the null stream), bit for
 * bit.  The call allocates nothing: it uses the model's resident state and the box's
 * phase tables, which dsx_set_grid prepares, and a device scratch array of
 * DSX_NOALLOC_SCRATCH_BYTES bytes, one per device, held from the first call on that
 * device until the process ends, for the spectra and partial lattice sums
 * (spectrum_bytes + the partial sums, each rounded up to 256 bytes, of
 * dsx_plan_query's model; every byte is written before it is read, so nothing is
 * cleared).  Every call on a device shares that device's scratch: calls that overlap
 * on one device (different streams, or threads) race and must be serialised by the
 * caller.  The model's own spectra are left stale (the next dsx_compute_intensity
 * recomputes them).  Errors: DSX_ERR_UNSUPPORTED when the spectra and partial sums
 * exceed the scratch; DSX_ERR_STATE when sites or grid are missing or the grid's
 * tables are not resident (dsx_compute_intensity then reports why); DSX_ERR_ARG when
 * the current device is not the model's.  With dsx_profile_enable on, the
 * instrumentation creates HIP events.
 */
#define DSX_NOALLOC_SCRATCH_BYTES (96 * 1024 * 1024)
dsx_status dsx_compute_intensity_noalloc(dsx_model m, float* out, void* hip_stream);

/*
 * Lanczos resampling of I on the box (Sec. V.B, Eqs. intensity_convol_finite,
 * windowed_sinc, lanczos): I(Q) = sum_G I(G) W(Q-G) / sum_G W(Q-G), W the product
 * over axes of sinc(2 pi r_cut d) sinc(pi d/m) for |d| < m, r_cut = (1 - 1/m)/2,
 * summed over floor(Q_a) - m + 1 <= G_a <= floor(Q_a) + m.  I(G) is computed
 * internally on the box grown by the window (no clamping or wrapping).
 * Output points Q_a = g0_a + i_a / s, i_a < s count_a; out float32
 * [s count0][s count1][s count2], same `where` / stream rules as above.
 * lanczos_m >= 2, oversample s >= 1.
 */
dsx_status dsx_noise_filter(dsx_model m, int32_t lanczos_m, int32_t oversample, float* out,
                            int32_t where, void* hip_stream);

/*
 * The same resampling with the cutoff modification of Sec. V.B (the second of the
 * three modifications listed after Eq. lanczos): r_cut = (1 - 1/m)/m' in Eq.
 * weight_sinc and m replaced by m m'/2 in Eq. lanczos, so that the idealized
 * real-space cutoff reaches 0 at |dr| = 1/m' (stronger noise suppression).  The
 * window spans G_a in [floor(Q_a) - w + 1, floor(Q_a) + w], w = m m'/2, and I(G) is
 * computed on the box grown by w.  mprime = 2 is dsx_noise_filter.
 * Requires mprime >= 2, lanczos_m * mprime even (w whole) and w <= 16; output and
 * `where` / stream rules as for dsx_noise_filter.
 */
dsx_status dsx_noise_filter_cutoff(dsx_model m, int32_t lanczos_m, int32_t mprime, int32_t oversample,
                                   float* out, int32_t where, void* hip_stream);

/*
 * The same resampling with the spherically symmetric cutoff of Sec. V.B (the third
 * modification): Eq. weight_sinc replaced by W_r(|Q - G|), proportional to
 * sin(x)/x^3 - cos(x)/x^2 with x = |Q - G| r_c (Q - G Cartesian, inverse Angstrom),
 * r_c = (1 - 1/m) r_max and r_max the radius of the largest sphere inscribed in the
 * supercell; the window of Eq. lanczos is kept.  The weight is no longer separable:
 * every output sums its (2m)^3 neighbourhood.  Requires 2 <= lanczos_m <= 4 and
 * 1 <= oversample <= 4; output and `where` / stream rules as for dsx_noise_filter.
 */
dsx_status dsx_noise_filter_spherical(dsx_model m, int32_t lanczos_m, int32_t oversample, float* out,
                                     int32_t where, void* hip_stream);

/*
 * Lanczos resampling at arbitrary points Q (Sec. V.B; e.g. the off-axis (h h l)
 * planes of Sec. V.B, which a grid along the reciprocal axes cannot hold):
 * I(Q) = sum_G I(G) W(Q-G) / sum_G W(Q-G) over the (2w)^3 supercell Bragg points
 * G_a in [floor(Q_a) - w + 1, floor(Q_a) + w], w = m m'/2, with the weight of
 * dsx_noise_filter_cutoff (mprime = 2: the plain filter).  I(G) is computed on the
 * smallest box holding every window.
 *   q[npts][3]  host array, float64, Q in units of the supercell Bragg grid (the G
 *               of dsx_set_grid: G_a = n_a times the reciprocal-lattice index);
 *               finite, |Q_a| <= 1e6
 *   out[npts]   float32, host (where = DSX_HOST) or device memory
 * Returns when the result is complete (the call synchronises hip_stream).  Requires
 * lanczos_m >= 2, mprime >= 2, lanczos_m * mprime even and w <= 8.  The model's grid
 * itself is not used, but sites and a grid must be set (DSX_ERR_STATE otherwise).
 */
dsx_status dsx_filter_points(dsx_model m, int32_t lanczos_m, int32_t mprime, int64_t npts, const double* q,
                             float* out, int32_t where, void* hip_stream);

/*
 * Batched execution (an execution pattern; the arithmetic is that of
 * dsx_compute_intensity / dsx_noise_filter).  The paper prefers many small
 * supercells averaged as an ensemble (Sec. III.B) and notes that their intensity
 * calculations can run in parallel (Sec. VI).  A batch fixes a set of ready models
 * (sites and grid set), one device output per model and the filter parameters.
 * dsx_batch_create tunes and plans every model (dsx_autotune), then records each
 * model's launch sequence -- its lattice sums, FFTs, recombination, Bragg points and,
 * when lanczos_m >= 2, the filter -- and builds one hipGraph of kernel nodes from them.
 * In the merged form, the launches of one step that run the same kernel (same
 * template instance and block size) become one dispatch over a descriptor table:
 * model d's blocks take a range of the merged grid (aligned to the 8 XCDs) and read
 * their parameters from entry d, so models of uneven n share a dispatch wherever
 * their kernels do; kernels whose merged form would spill registers are not merged.
 * The per-model form gives every launch its own node.  A node waits only for the
 * nodes that hold its models' previous launches.  dsx_batch_run replays the graph on
 * hip_stream: one graph launch recomputes every model from its current sites
 * (dsx_set_sites between runs is allowed; grids and outputs are fixed).
 *   models[n]  distinct models; n >= 1
 *   lanczos_m  0 = unfiltered I(G) (outs[i]: [count0][count1][count2] of model i),
 *              >= 2 = filtered with oversample s (outs[i]: [s count0][s count1][s count2])
 *   outs[n]    device pointers, owned by the caller, alive while the batch is used
 * While a batch exists its models keep the buffers it recorded: dsx_set_grid,
 * dsx_destroy_model and a dsx_noise_filter whose grown box would need a larger
 * buffer return DSX_ERR_BUSY.  Other calls on the models stay allowed; every call
 * on a model, batch replays included, is ordered after the model's previous work
 * whatever stream it was on.
 */
typedef struct dsx_batch_s* dsx_batch;

dsx_status dsx_batch_create(const dsx_model* models, int32_t n, int32_t lanczos_m, int32_t oversample,
                            float* const* outs, dsx_batch* out);
/* mode of dsx_batch_create_mode: DSX_BATCH_AUTO builds both forms, times three
 * replays of each on the device and keeps the faster (what dsx_batch_create does) */
enum { DSX_BATCH_AUTO = 0, DSX_BATCH_PER_MODEL = 1, DSX_BATCH_MERGED = 2 };
dsx_status dsx_batch_create_mode(const dsx_model* models, int32_t n, int32_t lanczos_m, int32_t oversample,
                                 float* const* outs, int32_t mode, dsx_batch* out);
typedef struct {
    int32_t mode;              /* the form the batch runs: DSX_BATCH_PER_MODEL or DSX_BATCH_MERGED */
    int32_t launches;          /* kernel launches of all models' sequences */
    int32_t dispatches;        /* kernel nodes of the graph the batch replays */
    int32_t merged_nodes;      /* nodes of that graph that serve more than one model */
    int32_t unmerged_spill;    /* launches kept apart because their merged kernel spills */
    int32_t merged_form_dispatches; /* kernel nodes of the merged form when it was built
                                       (also when the batch runs the per-model form); else -1 */
    float per_model_ms;        /* best of three replays of each form, when both were timed; else -1 */
    float merged_ms;
} dsx_batch_info;
/* DSX_ERR_ARG for a NULL batch or info */
dsx_status dsx_batch_query(dsx_batch b, dsx_batch_info* info);
dsx_status dsx_batch_run(dsx_batch b, void* hip_stream);
dsx_status dsx_batch_destroy(dsx_batch b);

/*
 * Autotuner: times the kernel variants of a ready model for its key (kind, n,
 * sites, order, configurations, box, filter) -- the recombination form, the number
 * of fields per FFT plane block and the filter's plane segment -- and keeps the
 * fastest.  With DSX_TUNE_CACHE naming a file, choices are read from / appended to
 * it (one line per key), so a key is tuned once and then always gets the same plan.
 * Runs kernels on hip_stream and waits for them.
 */
dsx_status dsx_autotune(dsx_model m, int32_t lanczos_m, void* hip_stream);

/*
 * The plan choices a model runs with (tuned by dsx_autotune, else the defaults):
 *   choice[0]  recombination form (0 default for the problem, 2 class form, 3 without
 *              the folded form, 4 folded without k3 slices)
 *   choice[1]  FFT fields per plane block (0 = chosen from the problem size)
 *   choice[2]  filter output planes per block
 * *tuned = 1 when they come from dsx_autotune.  Host memory, owned by the caller.
 */
dsx_status dsx_tune_query(dsx_model m, int32_t choice[3], int32_t* tuned);

/*
 * FFT knobs of a model (Sec. IV: the supercell FFTs): the radix sequence of each axis's
 * Stockham passes and the number of columns per block of the axis-1 transform in LDS.
 * The autotuner times every order of every grouping of the edge's factor 2^a into 4s
 * and 2s with its odd factors (at most 12 sequences per axis, the default first) on the
 * axes the LDS kernels transform -- edges 8, 16 and 32 take register kernels of a
 * fixed order -- and the tiles 16, 32 and 64; the choices join the tune cache line.
 *   radices   [3][16] int32, per axis the radices in pass order, 0-terminated; each
 *             2, 4 or odd (>= 3), product the edge n of the axis; NULL keeps the plans
 *   col_tile  0 (by edge: 64 up to n1 = 64, else 32), 16, 32 or 64
 * dsx_tune_set_fft marks the model tuned and its spectra stale.  DSX_ERR_ARG for an
 * invalid sequence or a tile whose LDS (8 n1 (1 + 2 tile) bytes) exceeds 160 KiB.
 * dsx_tune_query_fft writes the current sequences (0-padded) and tile.
 */
dsx_status dsx_tune_set_fft(dsx_model m, const int32_t* radices, int32_t col_tile);
dsx_status dsx_tune_query_fft(dsx_model m, int32_t* radices, int32_t* col_tile);

/*
 * Set the plan choices (same meaning as dsx_tune_query; the filter planes per block
 * in 1..64, forms 2-4 on nuclear models only) without timing anything, e.g. to
 * re-run a plan that dsx_autotune chose in another process.  The model then counts
 * as tuned.  Affects later calls, not batches already recorded.  DSX_ERR_ARG for a
 * value outside those sets; host memory, read only.
 */
dsx_status dsx_tune_set(dsx_model m, const int32_t choice[3]);

/*
 * Serving (an execution pattern; the arithmetic is that of dsx_compute_intensity /
 * dsx_noise_filter).  Refinement recomputes the intensity of a model again and
 * again as its variables change (Sec. I; Sec. VI), so a server keeps models
 * resident on the device -- plan, site variables, lattice sums and phase tables --
 * and runs requests with continuous batching: up to `slots` requests are on the
 * device at once, each on its own stream, and a request that arrives while others
 * run starts as soon as a slot and workspace are free.  A request's workspace --
 * the model's spectra, its partial lattice sums and, when filtered, the grown box
 * -- is taken from one device arena allocated at dsx_server_create; a request is
 * admitted only when its workspace fits in the free part of the arena (admission
 * by HBM footprint), and requests of one model run one after another in
 * submission order.  Waiting requests are served first come first served, except
 * that a request that fits may start before an earlier one that does not yet fit
 * (at most 64 times for one waiting request).  When several small requests (up to
 * 2^20 output voxels) can start at once, the dispatcher forms a round of up to
 * max_round of them on one slot (a larger request runs alone on its slot): each
 * request's site copy is issued as such, and the launches of all its steps run as
 * merged kernels (the form of dsx_batch_create_mode's merged graph, one kernel per step
 * and kernel instance over a descriptor table of the round's requests, issued directly
 * on the slot's stream with the tables copied from host memory pinned at creation);
 * the round's requests finish together.
 *   slots           1..16 rounds (of one or more requests) on the device at once
 *   queue_capacity  >= 1 requests waiting for admission; beyond it submit returns
 *                   DSX_ERR_BUSY
 *   arena_bytes     device workspace shared by requests on the device
 *   max_round       requests per round: 0 = 16, 1 = one request per slot (no merged
 *                   launches), at most 64
 */
typedef struct dsx_server_s* dsx_server;

typedef struct {
    int32_t slots;
    int32_t queue_capacity;
    int64_t arena_bytes;
    int32_t max_round;
} dsx_server_config;

/*
 * One request: replace the site variables of `config` (when config >= 0; the
 * pointers follow dsx_set_sites and must stay valid until the request finishes),
 * then compute I(G) on the model's grid (lanczos_m = 0) or the filtered intensity
 * (lanczos_m >= 2, oversample s >= 1) into the device array `out`
 * ([count0][count1][count2], or s times that per axis), owned by the caller.
 */
typedef struct {
    dsx_model model;
    int32_t config;
    const float* occ;
    const float* disp;
    const float* spin;
    int32_t where;
    int32_t lanczos_m;
    int32_t oversample;
    float* out;
} dsx_request;

/* Latencies are completion minus submission, over requests finished since the
 * last reset; voxels counts their output voxels. */
typedef struct {
    int64_t submitted, completed, failed, rejected;
    int64_t voxels;
    double p50_ms, p99_ms, mean_ms, max_ms;
    double span_s;             /* first submission to last completion */
    int64_t arena_bytes, arena_peak_bytes;
    int32_t slots, peak_in_flight;
    int64_t rounds;            /* rounds started (a round of one is a plain request) */
    int64_t round_requests;    /* requests they held */
} dsx_server_stats;

dsx_status dsx_server_create(const dsx_server_config* c, dsx_server* out);

/* A resident model owned by the server (dsx_create_model otherwise): set its grid
 * and sites with dsx_set_grid / dsx_set_sites (DSX_ERR_BUSY while it has requests
 * queued); direct compute calls on it return DSX_ERR_STATE. */
dsx_status dsx_server_add_model(dsx_server s, const dsx_model_desc* d, dsx_model* out);

/* Queue a request; *ticket identifies it.  DSX_ERR_BUSY: queue full.
 * DSX_ERR_NOMEM: the request's workspace exceeds the whole arena. */
dsx_status dsx_server_submit(dsx_server s, const dsx_request* r, int64_t* ticket);

/* Wait up to timeout_ms (< 0: no limit) for a request.  Returns DSX_OK once it
 * has finished, with its own status in *result (the ticket is then retired), or
 * DSX_ERR_BUSY if it is still queued or running.  Any thread may wait. */
dsx_status dsx_server_wait(dsx_server s, int64_t ticket, int32_t timeout_ms, dsx_status* result);

dsx_status dsx_server_stats_read(dsx_server s, int32_t reset, dsx_server_stats* out);

/* Finish every queued request, then release the server and its models. */
dsx_status dsx_server_destroy(dsx_server s);

/* Release a model and all its device memory (waits for its pending work).
 * DSX_ERR_BUSY while a batch still holds the model. */
dsx_status dsx_destroy_model(dsx_model m);

/* Message for the last failed call on this thread ("" if none). Never NULL. */
const char* dsx_last_error(void);

/*
 * Per-kernel timing (instrumentation; not part of the method).  While enabled,
 * every kernel the library launches (or each of the kind dsx_profile_select
 * names) is bracketed by two HIP events recorded on the stream it runs on.  dsx_profile_read waits for the recorded events, folds
 * them into per-kernel totals and copies at most `max` entries into `out`,
 * returning the number of kernel kinds seen since the last reset.  Process-wide;
 * safe to call from any thread.
 */
typedef struct {
    char    name[32];      /* "sums", "fft_planes", "fft_axis1", "recombine", "bragg", "lanczos" */
    int64_t launches;
    double  total_ms;
} dsx_kernel_stat;

dsx_status dsx_profile_enable(int32_t on);
/* Restrict the timing to one kernel kind (`kernel` one of the names above; the
 * other launches get no events, so they run as they do unprofiled), or time every
 * kind again with NULL or "".  DSX_ERR_ARG for a name longer than 31 bytes; a
 * name no kernel has simply times nothing. */
dsx_status dsx_profile_select(const char* kernel);
int32_t    dsx_profile_read(dsx_kernel_stat* out, int32_t max);
dsx_status dsx_profile_reset(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t dsx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DSX_H */
