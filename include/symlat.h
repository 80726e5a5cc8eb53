/*
 * symlat.h -- C ABI of the MI355X (gfx950) symplectic FRW lattice library.
 *
 * The library advances interacting real scalar fields phi_i(x), i = 1..N_f,
 * on a periodic n^3 comoving lattice in a self-consistently expanding
 * flat FRW background in conformal time, with the symplectic method of
 * Sainio, "PyCOOL - a Cosmological Object-Oriented Lattice code written in
 * Python" (arXiv:1201.5029):
 *
 *   - discretised Hamiltonian with the 7-point Laplacian member of the
 *     stencil family of Sec. 2.1, eq. (2.7), and radiation/matter terms,
 *     eq. (2.20);
 *   - three-way split H = H1 + H2 + H3 with exact flows, eq. (2.46)-(2.47);
 *   - second-order map eq. (2.48) composed to 4th order by the triple jump
 *     eq. (2.43)-(2.44), or to 6th/8th order with the symmetric
 *     compositions of eq. (2.45) and Table 1.
 *
 * Conventions shared by every entry point:
 *   - Every call returns sl_status; no exception crosses the ABI.  On error
 *     sl_last_error() returns a thread-local message (valid until the next
 *     call on that thread).
 *   - A lattice handle owns all of its device memory.  Host buffers passed
 *     in or out are owned by the caller and only read/written during the
 *     call.
 *   - Field arrays exchanged with the host are FP64, laid out
 *     [field][z][y][x] with x fastest: element (i, z, y, x) is at
 *     ((i*n + z)*n + y)*n + x.
 *   - Work is enqueued on the handle's HIP stream.  sl_evolve returns
 *     without waiting; device-side failures (non-finite lattice sums) are
 *     reported by the next synchronising call (sl_energies, sl_get_fields,
 *     sl_get_background, sl_spectrum, sl_synchronize) as SL_E_NONFINITE.
 *   - One handle must not be used from two threads at once (a batch and
 *     its members count as one).  Different handles may be used from
 *     different threads; the process-wide memory of tuned shapes is locked.
 */
#ifndef SYMLAT_H
#define SYMLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sl_lattice sl_lattice;
typedef struct sl_batch sl_batch;

typedef enum {
  SL_OK = 0,
  SL_E_INVALID = 1,   /* bad argument: nothing was changed                   */
  SL_E_NOMEM = 2,     /* device or host allocation failed                    */
  SL_E_DEVICE = 3,    /* a HIP runtime call failed                           */
  SL_E_STATE = 4,     /* call out of order (e.g. evolve before a potential)  */
  SL_E_NONFINITE = 5, /* a lattice sum or the background became non-finite   */
  SL_E_UNSTABLE = 6   /* omega_max*|dt| beyond the composition's stability   */
} sl_status;

/* Storage precision of phi and pi.  SL_FP32 stores and updates the fields
 * in FP32; the scale factor, its momentum, every stage coefficient and all
 * lattice sums stay FP64 with compensated (TwoSum) accumulation. */
typedef enum { SL_FP64 = 0, SL_FP32 = 1 } sl_precision;

/* SL_EXPAND_SELF: a and p_a follow eq. (2.47).  SL_EXPAND_NONE: static
 * background, a stays at a0 (H1 is the identity and p_a is not updated). */
typedef enum { SL_EXPAND_NONE = 0, SL_EXPAND_SELF = 1 } sl_expansion;

/* Potential families (Sec. 3 models in program units) and their params:
 *   SL_POT_FREE       (m_1^2, ..., m_Nf^2)   V = sum_i m_i^2 phi_i^2 / 2
 *   SL_POT_CHAOTIC2   (m^2, G)               V = m^2 phi^2/2 + G phi^2 chi^2/2
 *                                            (N_f = 2, Sec. 3.1, G = g^2)
 *   SL_POT_OSCILLON   (m^2, lambda, g)       V = m^2 phi^2/2 - lambda phi^4/4
 *                                                + g phi^6/6   (N_f = 1)
 *   SL_POT_QBALL_LOG  (m^2, K, M^2)          u = (phi_1^2 + phi_2^2)/2,
 *                                            V = m^2 u (1 + K ln(u/M^2)),
 *                                            V = dV = 0 at u = 0 (N_f = 2,
 *                                            Sec. 3.3 without |Phi|^6)    */
typedef enum {
  SL_POT_FREE = 0,
  SL_POT_CHAOTIC2 = 1,
  SL_POT_OSCILLON = 2,
  SL_POT_QBALL_LOG = 3
} sl_potential;

/* Initial fluctuations added to the homogeneous values:
 *   SL_FLUCT_NONE    none
 *   SL_FLUCT_VACUUM  Gaussian field with E|f_n|^2 = A^2/(2 omega_n L^3),
 *                    omega_n^2 = k_eff^2/dx^2 + d2V/dphi_i^2 (homogeneous
 *                    point), k_eff^2 = sum_d 4 sin^2(pi n_d/n), zero mode
 *                    removed, built in k-space and inverse transformed
 *   SL_FLUCT_WHITE   i.i.d. N(0, A^2) per site with its lattice mean removed
 * Normal deviates come from a counter-based SplitMix64 + Box-Muller
 * generator keyed by (seed, field, index, component), so the draw does not
 * depend on launch shape. */
typedef enum { SL_FLUCT_NONE = 0, SL_FLUCT_VACUUM = 1, SL_FLUCT_WHITE = 2 } sl_fluct;

typedef struct {
  int32_t n;         /* lattice side, 4 <= n <= 1024                        */
  int32_t nfields;   /* N_f, 1..8                                           */
  double L;          /* comoving side length (> 0); dx = L/n                */
  int32_t precision; /* sl_precision                                        */
  int32_t expansion; /* sl_expansion                                        */
  double mpl;        /* reduced Planck mass m_pl (> 0)                      */
  double a0;         /* initial scale factor (> 0)                          */
  double rho_rad0;   /* homogeneous radiation V_L rho_gamma0 term, eq. (2.20) */
  double rho_mat0;   /* homogeneous matter term, eq. (2.20)                 */
} sl_config;

/* Observables of eq. (2.16), (2.18), (3.1) at the current time, computed on
 * the device at the synchronised state (pending field drifts applied
 * virtually; the stored state is not modified). */
typedef struct {
  double eta;                /* conformal time                                  */
  double a, p_a;             /* scale factor and its momentum                    */
  double hubble;             /* H = a'/a^2 = -p_a/(6 V_L m_pl^2 a^2); 0 if static */
  double rho, pressure;      /* <rho>, <P> of the fields, eq. (2.16)             */
  double w_eos;              /* <P>/<rho>                                         */
  double friedmann_residual; /* |<rho_tot>/(3 m_pl^2 H^2) - 1|, eq. (3.1); NaN if static */
  double h_total;            /* total Hamiltonian eq. (2.20) (no H1 term if static) */
  double pot;                /* <V>                                               */
  double kin[8];             /* <pi_i^2>/(2 a^6)                                   */
  double grad[8];            /* <G[phi_i]>/(2 a^2 dx^2), eq. (2.8)                 */
  double mean[8];            /* <phi_i>                                            */
  double var[8];             /* <phi_i^2> - <phi_i>^2                              */
} sl_energies_t;

/* Create a lattice (Sec. 2.1 state: phi, pi, a, p_a).  hip_stream is a
 * hipStream_t owned by the caller or NULL (the handle then creates its own
 * non-blocking stream).  Allocates device memory for two copies of (phi,
 * pi) in the storage precision plus O(#blocks) FP64 partial sums.
 * SL_E_INVALID for n < 4 or n > 1024, nfields outside 1..8, L, mpl or a0
 * not > 0, or a NULL argument. */
sl_status sl_lattice_create(const sl_config* cfg, void* hip_stream, sl_lattice** out);

/* As sl_lattice_create, but the handle adopts the caller's four field
 * arrays instead of allocating them: phi0, pi0 (buffer 0) and phi1, pi1
 * (buffer 1), each nfields * n^3 elements of the storage precision in the
 * device layout [z][field][y][x] (the fields of each z-plane one after the
 * other: element (i, z, y, x) at ((z*nfields + i)*n + y)*n + x; host arrays
 * keep [field][z][y][x]), in device memory of the current device (hipMalloc
 * or a pool carved from it), 16-byte aligned and not overlapping.  The
 * handle zero-fills them at creation, uses them until sl_lattice_destroy and
 * never frees them; the caller keeps them alive that long and touches them
 * only between synchronising calls.  Which buffer holds the state alternates
 * with the stages, and in FP32 storage the arrays hold each field's and
 * momentum's remainder around a homogeneous FP64 offset the handle keeps:
 * read the state with sl_get_fields.  The small buffers (partial
 * sums, scalars) are still the handle's.  SL_E_INVALID if an array is NULL,
 * misaligned, not device memory of this device, shorter than needed inside
 * its allocation, or overlaps another.  sl_footprint_bytes still counts the
 * four arrays. */
sl_status sl_lattice_create_with_buffers(const sl_config* cfg, void* hip_stream, void* phi0,
                                         void* pi0, void* phi1, void* pi1, sl_lattice** out);

/* Release all device memory of the handle; NULL is a no-op. */
sl_status sl_lattice_destroy(sl_lattice* lat);

/* Select the potential family and copy its nparams parameters (see
 * sl_potential; the models of Sec. 3.1-3.3).  SL_E_INVALID if the family
 * does not fit nfields or nparams is wrong.  Must precede
 * sl_init_fluctuations / sl_evolve.  A batch member may take new
 * parameters of its family (its next batched step uses them; its tile is
 * kept); SL_E_STATE if it is given another family. */
sl_status sl_set_potential(sl_lattice* lat, int32_t kind, const double* params, int32_t nparams);

/* Discrete Laplacian of eq. (2.7), from the cubic family the paper draws
 * its second-order stencils from: c[0] weights the site, c[1] its 6 face,
 * c[2] its 12 edge and c[3] its 8 corner neighbours; G of eq. (2.8) uses
 * the same weights, G = 1/2 sum_nbr c_class (f(nbr) - f(x))^2.  The default
 * is the 7-point member (-6, 1, 0, 0).  A member must annihilate constants
 * (c0 + 6 c1 + 12 c2 + 8 c3 = 0) and tend to the Laplacian (c1 + 4 c2 +
 * 4 c3 = 1); its leading error is isotropic when c1 = 2 c2 + 8 c3, e.g.
 * the 19-point (-4, 1/3, 1/6, 0) and 27-point (-128/30, 14/30, 3/30, 1/30)
 * members.  Any member other than the 7-point one runs the 27-point pass
 * (vx = 1 or 2 sites per lane, pf = 1, or pf = 5 with vx = 2).  The stencil enters the kick, the
 * p_a sums, the observables, the stability bound (largest k_eff^2 over the
 * zone) and the vacuum mode frequencies, so set it before
 * sl_init_fluctuations.  c is a host array of 4 doubles.  SL_E_INVALID for
 * non-finite values or a member outside the family (tolerance 1e-12 of the
 * weighted coefficient sum); SL_E_STATE for a change of stencil kind while
 * the lattice belongs to a batch.  sl_get_stencil copies the weights out. */
sl_status sl_set_stencil(sl_lattice* lat, const double* c);
sl_status sl_get_stencil(sl_lattice* lat, double* c_out);

/* Initial state: phi_i = phi0[i] + fluctuation, pi_i = pi0[i] (canonical
 * momenta), a = a0, eta = 0, then p_a from the constraint H = 0 on the
 * expanding branch (p_a < 0), eq. (2.20).  phi0 and pi0 hold nfields
 * doubles.  amplitude is A of sl_fluct.  Runs entirely on the device.
 * SL_E_INVALID for an unknown kind, a negative amplitude, or VACUUM where
 * a field's effective mass is undefined; SL_E_STATE if the constraint has
 * no real solution. */
sl_status sl_init_fluctuations(sl_lattice* lat, const double* phi0, const double* pi0,
                               int32_t kind, double amplitude, uint64_t seed);

/* Advance `steps` composed steps of size dt (dt < 0 runs backwards) with
 * the given order: 2 (eq. (2.48)), 4 (triple jump, eq. (2.43)), 6 or 8
 * (Table 1).  Each stage is one fused device pass (drift owed from the
 * previous H2 flows, Laplacian, kick, FP64 block sums) and one device-side
 * scalar update, run by the next pass itself where passes chain (see
 * sl_set_chaining) or by a one-workgroup kernel; the trailing field drift
 * of the last stage is kept pending, so evolve(a) then evolve(b) equals
 * evolve(a + b) bit for bit.
 * Interior chunks of 32 steps replay a HIP graph captured on first use (the
 * same launches as the eager path; recaptured when dt, order or the launch
 * shape change); the final 1..32 steps and timed calls launch eagerly.
 * SL_E_INVALID for steps < 0, dt not finite, or an unknown order;
 * SL_E_UNSTABLE if omega_max |dt| exceeds the order's linear stability
 * limit (omega_max^2 = k_eff,max^2/dx^2 + a^2 max(m_eff^2, 0), with
 * k_eff,max^2 = 12 for the 7-point stencil). */
sl_status sl_evolve(sl_lattice* lat, int64_t steps, double dt, int32_t order);

/* Compute the observables (one extra read pass over the lattice) and
 * copy them to *out; synchronises the stream. */
sl_status sl_energies(sl_lattice* lat, sl_energies_t* out);

/* Field power spectrum of phi_field (the spectra of the post-processing
 * step, Sec. 2.4; the field of the synchronised state, eq. (2.12)):
 * F_n = DFT(phi)/n^3, modes binned by
 * |n| rounded half away from zero (decided in integers), the n = 0 mode
 * excluded, modes with bin >= nbins dropped.  k_out[b] = 2 pi <|n|>_b / L,
 * p_out[b] = <|F_n|^2>_b, count_out[b] = number of modes; empty bins are
 * zero.  Host arrays of nbins entries; 1 <= nbins <= 2048.  Synchronises. */
sl_status sl_spectrum(sl_lattice* lat, int32_t field, int32_t nbins,
                      double* k_out, double* p_out, int64_t* count_out);

/* sl_spectrum for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and outputs, with the transform buffers and
 * binning partials in a library-owned static device array of 32 MiB per
 * GPU (held until the process ends) instead of per-call allocations.
 * Accepts lattices whose scratch fits it: 32 n^3 + 16 n bytes of transform
 * buffers and twiddles (rounded up to 256) plus 24 nbins m bytes of binning
 * partials, m = min(ceil(n^3 / 256), 256) -- e.g. n <= 86 with any nbins,
 * n = 96 with up to 853 bins, n <= 101 with a few bins.  Every call on one GPU shares that array, so calls that
 * overlap on one GPU (two threads, or two streams without an ordering
 * between them) race; the array keeps the last call's contents and each
 * call writes all it reads.  SL_E_INVALID beyond the limit (with the
 * bytes needed in sl_last_error) and as sl_spectrum otherwise; allocates
 * no device memory.  Synchronises. */
sl_status sl_spectrum_noalloc(sl_lattice* lat, int32_t field, int32_t nbins, double* k_out,
                              double* p_out, int64_t* count_out);

/* Field, energy-density and number-density spectra of phi_field (the
 * post-processing spectra of Sec. 2.4), from F_n = DFT(phi)/n^3 and
 * P_n = DFT(pi)/n^3 of the synchronised state, k_eff^2 of the lattice's
 * stencil and m_eff^2 = the lattice mean of d^2V/dphi_field^2:
 *   rho_n = |P_n|^2/(2 a^6) + (k_eff^2/(2 a^2 dx^2) + m_eff^2/2) |F_n|^2,
 *   n_n = rho_n / omega_n, omega_n^2 = k_eff^2/(a^2 dx^2) + m_eff^2
 *   (n_n = 0 where omega_n^2 <= 0).
 * Binned as sl_spectrum; per bin the means of |F_n|^2 (pf_out), rho_n
 * (pe_out) and n_n (pn_out), k_out and count_out as sl_spectrum; *m2eff_out
 * (may be NULL) receives m_eff^2.  The sum of count * pe over all bins is
 * the fluctuations' kinetic, gradient and m_eff^2 energy density.  Host
 * arrays of nbins entries; 1 <= nbins <= 2048.  Synchronises. */
sl_status sl_spectra(sl_lattice* lat, int32_t field, int32_t nbins, double* k_out,
                     double* pf_out, double* pe_out, double* pn_out, int64_t* count_out,
                     double* m2eff_out);

/* Copy the synchronised state -- the lattice fields phi_i and their
 * canonical momenta pi_i = a^2 phi_i' (eq. (2.12)), the field variables of
 * the Hamiltonian (2.13), with any pending field drift applied -- to
 * caller-owned host FP64 arrays of nfields*n^3 each, layout [field][z][y][x]
 * (either pointer may be NULL).  SL_E_NOMEM if the device staging buffer
 * cannot be allocated.  Synchronises. */
sl_status sl_get_fields(sl_lattice* lat, double* phi_out, double* pi_out);

/* Replace the state (phi_i, pi_i of eq. (2.12)) by caller-owned host
 * FP64 arrays of nfields*n^3 each, layout [field][z][y][x] (rounded to the
 * storage precision), set a, eta = 0 and p_a; p_a = NaN means "solve the
 * constraint that the Hamiltonian (2.13) vanishes" (the first Friedmann
 * equation (2.18); expanding branch, p_a < 0).  A potential must be
 * set.  SL_E_INVALID for NULL arrays or a <= 0; SL_E_STATE without a
 * potential; SL_E_NONFINITE if the state is not finite or the constraint
 * has no real p_a. */
sl_status sl_set_fields(sl_lattice* lat, const double* phi, const double* pi,
                        double a, double p_a);

/* Background history (for the uniform-density Delta N of a scan over
 * initial values, Sec. 2.4 and Sec. 4): with capacity > 0, every completed
 * step (alone or in a batch) appends (eta, a, p_a, rho) at its end to a
 * device buffer of that many records (further steps are not recorded);
 * capacity 0 releases it.  rho is the total density on that time slice from
 * the first Friedmann equation (2.18): rho = 3 m_pl^2 H^2 with the Hubble
 * rate H = a'/a^2, a' = -p_a / (6 V_L m_pl^2) (eq. (2.14));
 * 0 in a static background.  The record restarts at 0 entries here and
 * whenever the state is reset (sl_init_fluctuations, sl_set_fields).
 * sl_get_history copies up to cap records into four host arrays of cap
 * entries (caller-owned; all four non-NULL when a record is copied) and
 * reports the number recorded in *count.  SL_E_NOMEM if the buffer cannot
 * be allocated (the lattice then records nothing).  Synchronises. */
sl_status sl_set_history(sl_lattice* lat, int64_t capacity);
sl_status sl_get_history(sl_lattice* lat, double* eta, double* a, double* p_a, double* rho,
                         int64_t cap, int64_t* count);

/* Conformal time, scale factor and its momentum.  Synchronises. */
sl_status sl_get_background(sl_lattice* lat, double* eta, double* a, double* p_a);

/* Wait for the handle's stream; reports sticky device-side errors. */
sl_status sl_synchronize(sl_lattice* lat);

/* Device bytes a lattice of this configuration holds from creation to
 * destruction (0 if invalid); sl_set_history adds 32 bytes per record.
 * sl_transient_bytes: the most any single call on such a lattice allocates
 * on top while it runs and frees before returning (vacuum or white initial
 * state, sl_set_fields / sl_get_fields staging, sl_spectrum, sl_spectra);
 * 0 if invalid.  Admission keeps footprint + transient free. */
size_t sl_footprint_bytes(const sl_config* cfg);
size_t sl_transient_bytes(const sl_config* cfg);

/* Thread-local message of the last failing call on this thread. */
const char* sl_last_error(void);

/* Host helpers (no device work):
 * sl_composition_weights writes the s stage weights of `order` into w_out
 * (capacity cap) and returns s, or -1 for an unknown order / small cap;
 * sl_stability_limit returns the largest stable omega*h of the order's
 * composition on a harmonic mode, or -1. */
int32_t sl_composition_weights(int32_t order, double* w_out, int32_t cap);
double sl_stability_limit(int32_t order);

/* Kernel timing for measurement: while enabled, sl_evolve brackets every
 * fused stage pass with HIP events on the handle's stream.
 * sl_kernel_timing synchronises and returns the number of timed passes and
 * their summed duration (ms) since enabling, then clears the record. */
sl_status sl_set_kernel_timing(sl_lattice* lat, int32_t enable);
sl_status sl_kernel_timing(sl_lattice* lat, int64_t* passes, double* total_ms);

/* Launch shape of the fused pass: tx lanes along x (8 .. 64), each
 * holding vx consecutive x-sites (1, 2 or 4; n must be divisible by vx),
 * ty = floor(256/tx) rows (the remaining 256 - tx*ty lanes of the workgroup
 * idle), tz z-planes per workgroup, and the pass mode pf: the prefetch
 * depth of the z-march (1: next plane loaded each iteration; 2: own column
 * two planes and halo one plane ahead; 3: own column three planes and halo
 * two planes ahead, with non-temporal stores only), plus 4 to write the
 * results with non-temporal stores (so they do not displace halo data in
 * the L2; vx = 2 or 4 only), i.e. pf in {1, 2, 5, 6, 7}.
 * Lattices with more than two fields run with vx = 1, pf = 1; any stencil
 * other than the 7-point one runs with pf = 1 and vx = 1 or 2, or pf = 5
 * and vx = 2 (2 only up to two fields; 2 tx + 2 ty + 4 <= 256 halo lanes,
 * true for every tx).  A batch
 * member keeps its vx and pf.  sl_get_tile reports the shape in use; sl_set_tile
 * overrides it (tz = 0: z-chunk chosen from the kernel's occupancy so the
 * grid fills whole rounds of resident workgroups).  SL_E_INVALID for
 * unsupported shapes or more than 65536 workgroups. */
sl_status sl_get_tile(sl_lattice* lat, int32_t* tx, int32_t* vx, int32_t* ty, int32_t* tz,
                      int32_t* pf);
sl_status sl_set_tile(sl_lattice* lat, int32_t tx, int32_t vx, int32_t tz, int32_t pf);

/* Stage chaining of sl_evolve.  The scalar update that closes a stage
 * (the p_a kicks of eq. (2.14) with the lattice sums of the stage, and the
 * drift coefficient of the next) either runs as its own one-workgroup
 * kernel after each fused pass (mode 0), or is folded into the next pass
 * (mode 1): every workgroup of that pass reduces the previous pass's
 * per-tile sums and forms the same scalars before its z-march, and one
 * finalize kernel closes each captured chunk of steps.  Both modes give
 * bitwise identical fields, background and history.  Modes -1 (the
 * default) and 1 chain lattices with at most 1024 tiles (more run a
 * finalize after every pass); mode 0 never chains.  Batches do not chain.
 * SL_E_INVALID for other modes. */
sl_status sl_set_chaining(sl_lattice* lat, int32_t mode);

/* Autotuner: time candidate shapes (tx in {16, 32, 64}, 8 with vx = 4, and
 * n/vx when that is in [8, 64] and not a power of two, i.e. a whole row per
 * tile; vx in {1, 2, 4} dividing n; pf in {1, 2, 5, 6, 7}; tz in {occupancy choice,
 * n/16, n/8, n/4, n/2}, at least 8, and for n <= 128 also 1, 2 and 4)
 * on the lattice's current state: best of `reps` HIP-event timings of six
 * consecutive stages as sl_evolve runs them with that shape (chained
 * passes, or fused pass + finalize where the passes do not chain; each
 * reading what the previous wrote) with the drift and kick coefficients
 * frozen at zero, so the fields keep their values; the scalars are restored
 * after.  Before any timing the GPU is warmed up (0.1 s of frozen stages
 * in the current shape).  The three fastest (those within 5 % of the best)
 * are then timed again over 24 stages each, in max(reps, 3) rounds that
 * take them in rotating order, all enqueued back to back behind a warm-up
 * with no host wait between them, and the lowest mean wins.
 * best_ms is the time of one stage.  vx_only / pf_only
 * (0 = free) restrict the search; a batch member is tuned within its own vx
 * and pf (the batch is rebuilt at its next step).
 * The winner is applied and remembered for this process: lattices created
 * later with the same (device, n, fields, precision, potential family) start
 * with it.  Outputs may be NULL.  sl_autotune_forget clears that memory and
 * the batch tuner's. */
sl_status sl_autotune(sl_lattice* lat, int32_t reps, int32_t vx_only, int32_t pf_only,
                      int32_t* tx, int32_t* vx, int32_t* tz, int32_t* pf, double* best_ms);
sl_status sl_autotune_forget(void);

/* Batched form: many lattices advanced together, as in the ensemble of
 * runs with different initial values that the separate-universe
 * calculation needs (Sec. 2.4, Sec. 4).  Members share storage precision,
 * potential family, field count and stencil kind; sizes, parameters, tile
 * widths and z-chunks may differ.  A joining lattice takes the batch's
 * per-lane shape (vx, pf) of the fused pass (its tx and z-chunk are reset,
 * or set from the batch tuner's record for its size).  Each
 * stage is one fused pass over the concatenated tiles of all members (each
 * XCD strides through a contiguous range of them) and one finalize with a
 * workgroup per member; interior chunks of 8 steps of a call replay one
 * captured HIP graph (kept while dt, order and membership are unchanged,
 * whatever the step count), the last 1 .. 8 steps launch eagerly.  A member's
 * result is bit-identical to evolving it alone with the same tile shape.
 * The batch does not own its members: destroying a lattice removes it.
 * hip_stream: caller-owned hipStream_t or NULL (own stream).  The batch
 * orders itself after each member's stream and each member's stream after
 * the batch.  SL_E_INVALID for a mismatched or duplicate member. */
sl_status sl_batch_create(void* hip_stream, sl_batch** out);
sl_status sl_batch_destroy(sl_batch* batch);
sl_status sl_batch_add(sl_batch* batch, sl_lattice* lat);
sl_status sl_batch_remove(sl_batch* batch, sl_lattice* lat);
sl_status sl_batch_count(const sl_batch* batch, int32_t* count);
/* Workgroups of the batched pass.  0 (the default) launches one per tile,
 * and the dispatcher balances tiles of different sizes over the CUs;
 * w > 0 launches min(w, tiles) workgroups that stay resident and stride
 * through the concatenated tile list, each XCD through a contiguous range
 * (the persistent form).  Results are the same bit for bit either way.
 * sl_batch_autotune sets it.  sl_batch_get_grid reports the request and the
 * workgroup count the next step launches (0 for an empty batch); outputs
 * may be NULL.  SL_E_INVALID for w < 0 or w > 2^24. */
sl_status sl_batch_set_grid(sl_batch* batch, int32_t workgroups);
sl_status sl_batch_get_grid(const sl_batch* batch, int32_t* requested, int32_t* launched);
/* Advance every member `steps` steps (same dt and order for all). */
sl_status sl_batch_step(sl_batch* batch, int64_t steps, double dt, int32_t order);
/* Batch autotuner: after a warm-up of the GPU (0.1 s of the batched pass
 * in the current shapes), every per-lane shape (vx in {1, 2, 4} dividing all
 * member sizes, pf in {1, 2, 5, 6, 7}, as the field count and stencil allow) is timed
 * at starting shapes (a whole row per tile, at most 64 lanes, quarter-lattice
 * z-chunks); for the three fastest, per member size (largest share
 * of sites first, two rounds of coordinate descent) the same tx candidates
 * as sl_autotune and
 * z-chunks n/{1, 2, 4, 8} (and n/3, n/6 where they divide n) are tried for
 * all members of that size, timing
 * the batched pass alone (best of `reps`
 * HIP-event timings of four consecutive passes; the members' states are
 * left unchanged), and keep a shape only if it is at least 1 % faster,
 * and again when the two are timed one right after the other (a later lane
 * shape replaces an earlier one likewise); last,
 * with the chosen shapes, the persistent grid of the resident capacity is
 * timed against one workgroup per tile and kept only if 0.5 % faster (see
 * sl_batch_set_grid).  The chosen shapes are applied to the members
 * (also for their own sl_evolve calls) and remembered for this process:
 * lattices of a tuned size that join a batch later are given that shape.
 * best_ms (may be NULL) receives the final pass time.  SL_E_STATE for an
 * empty batch. */
sl_status sl_batch_autotune(sl_batch* batch, int32_t reps, double* best_ms);
/* Time the batched pass with the members' current shapes, as the batch
 * autotuner times a candidate (best of `reps` HIP-event timings of four
 * consecutive passes; the members' states are left unchanged): *ms = one
 * pass.
 * SL_E_STATE for an empty batch. */
sl_status sl_batch_time_pass(sl_batch* batch, int32_t reps, double* ms);
/* Wait for the batch and report members' sticky device errors. */
sl_status sl_batch_synchronize(sl_batch* batch);

/* Free and total device memory (for admission by sl_footprint_bytes). */
sl_status sl_device_memory(size_t* free_bytes, size_t* total_bytes);

/* Measurement helper: time `iters` plain device-to-device copies of `bytes`
 * bytes (bytes a multiple of 16, >= 1024; one 16-byte element per lane) on a
 * private stream and return the
 * achieved read+write bandwidth in GB/s.  Used to calibrate memory counters
 * and to state the achievable HBM bandwidth beside the lattice kernels. */
sl_status sl_hbm_copy_bench(size_t bytes, int32_t iters, double* gbs);

/* ---------------------------------------------------------------------------
 * Linearized integrator (Sec. 2.2 and Sec. 2.4).  The fields are a
 * homogeneous background phi0_i (momentum pi0_i = a^2 phi0_i' per site) plus
 * perturbations with zero lattice sum, eq. (2.21)-(2.22); the Hamiltonian is
 * kept to second order in the perturbations, eq. (2.34), which do not act
 * back on a, p_a or the background.  A step composes the second-order map
 * of eq. (2.50) over the five parts of eq. (2.49) with the weights of
 * sl_evolve's orders.  The perturbations are evolved in Fourier space, eq.
 * (2.38): every mode class with the same k_eff^2 (modes whose folded wave
 * numbers min(n_d, N - n_d) form the same multiset) is integrated once as
 * growth functions, the 2N x 2N matrix M of eq. (2.51), which then advances
 * every Fourier mode of the class.  FP64 throughout; at most 4 fields.
 * ------------------------------------------------------------------------- */
typedef struct sl_linear sl_linear;

/* Create a handle for cfg (precision must be SL_FP64, nfields <= 4); the
 * stream is as for sl_lattice_create.  Device memory: 4 nfields n^3
 * complex modes plus transform scratch, and (2 nfields)^2 doubles per
 * mode class (C(n/2 + 3, 3) classes).  SL_E_INVALID for a bad config. */
sl_status sl_linear_create(const sl_config* cfg, void* hip_stream, sl_linear** out);
sl_status sl_linear_destroy(sl_linear* lin);
/* Potential family and parameters, as sl_set_potential. */
sl_status sl_linear_set_potential(sl_linear* lin, int32_t kind, const double* params,
                                  int32_t nparams);
/* Laplacian weights (centre, face, edge, corner), as sl_set_stencil; the
 * stencil sets k_eff^2 of every mode. */
sl_status sl_linear_set_stencil(sl_linear* lin, const double* c);
/* State from host FP64 lattice fields phi, pi (nfields n^3 each, [field][z]
 * [y][x]): phi0_i, pi0_i are their lattice means, the perturbations the
 * remainders, transformed to Fourier space on the device (the k = 0 mode
 * set to zero).  a = a0, eta = 0; p_a = NaN solves the background
 * constraint H1 + H2 + H3 = 0 of eq. (2.49) on the expanding branch.
 * Synchronises. */
sl_status sl_linear_set_fields(sl_linear* lin, const double* phi, const double* pi, double p_a);
/* Advance `steps` composed steps of size dt: background coefficients per
 * stage, growth functions of every class, then every mode times its M.
 * Asynchronous.  SL_E_INVALID / SL_E_UNSTABLE as sl_evolve (stability from
 * the largest k_eff^2 and the Hessian diagonal at phi0). */
sl_status sl_linear_evolve(sl_linear* lin, int64_t steps, double dt, int32_t order);
/* Lattice fields phi0 + delta phi and pi0 + delta pi as host FP64 arrays
 * (inverse transform on the device); either pointer may be NULL.
 * Synchronises. */
sl_status sl_linear_get_fields(sl_linear* lin, double* phi_out, double* pi_out);
/* Background: conformal time, a, p_a and phi0, pi0 (nfields each; any
 * pointer may be NULL).  Synchronises. */
sl_status sl_linear_get_background(sl_linear* lin, double* eta, double* a, double* p_a,
                                   double* phi0, double* pi0);
/* Number of mode classes (distinct folded wave-number multisets). */
sl_status sl_linear_classes(sl_linear* lin, int64_t* nclasses);
sl_status sl_linear_synchronize(sl_linear* lin);
/* Measurement: while enabled, each evolve call brackets its background and
 * growth launches and its apply launch with HIP events on the handle's
 * stream; sl_linear_kernel_timing synchronises, returns the number of
 * growth launches and the summed growth, background and apply times (ms)
 * since the last call, and clears the record. */
sl_status sl_linear_set_kernel_timing(sl_linear* lin, int32_t enable);
sl_status sl_linear_kernel_timing(sl_linear* lin, int64_t* growth_launches, double* growth_ms,
                                  double* table_ms, double* apply_ms);

#ifdef __cplusplus
}
#endif

#endif /* SYMLAT_H */
