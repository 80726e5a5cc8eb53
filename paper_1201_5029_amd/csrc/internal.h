// Internal declarations shared by the HIP kernels and the host runtime of
// libsymlat (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "symlat.h"

namespace symlat {

// ---- host helpers shared by the runtime sources (runtime.hip) -------------
// Record the thread-local message of sl_last_error and return st.
sl_status fail(sl_status st, const char* fmt, ...);
// Stage weights of the order-2/4/6/8 composition (empty if unknown).
std::vector<double> weights_for(int order);
// Largest stable omega*h of the composition on a harmonic mode (-1 if unknown).
double stability_limit_for(int order);
// d^2 V / d phi_i^2 at a homogeneous point; false where undefined.
bool hessian_diag(int kind, int nf, const double* p, const double* f, double* out);
// Parameter count of a potential family (-1 if unknown) and the field count
// it requires (0: any).
int nparams_for(int kind, int nf);
int nfields_for(int kind);
bool config_ok(const sl_config* c, std::string* why);

#define HIP_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::symlat::fail(SL_E_DEVICE, "%s failed: %s", #expr,               \
                            hipGetErrorString(e_));                            \
  } while (0)

constexpr int kBlock = 256;     // threads per workgroup of every lattice kernel
constexpr int kMaxFields = 8;
constexpr int kMaxBins = 2048;
// Idle lanes of the fused pass store here: 256 threads x 2 arrays x 8 fields
// x 4 sites x 8 bytes.
constexpr size_t kSinkBytes = size_t(kBlock) * 2 * kMaxFields * 4 * 8;

// Doubles per background history record: eta, a, p_a, rho.
constexpr int kHistRecord = 4;

// Sticky device-side error bits in DevScalars::status.
constexpr int kStatusNonFinite = 1;

// Background scalars and the coefficients of the next fused pass, resident
// in device memory (FP64).  Only device kernels update them during
// evolution; the host reads them after a synchronisation.
struct DevScalars {
  double a;        // scale factor
  double p_a;      // its canonical momentum
  double eta;      // conformal time
  double S2;       // sum_{i,x} pi_i^2 of the stored momenta
  double c_pend;   // field drift owed: phi_true = phi_stored + c_pend * pi
  double c_next;   // drift the next pass applies before its kick
  double alpha;    // kick coefficient of the Laplacian: a^2 w h / dx^2
  double beta;     // kick coefficient of dV: a^4 w h
  double a_kick;   // scale factor during the next kick
  double S3_last;  // last H3 lattice sum (diagnostic)
  int32_t parity;  // which ping-pong buffer holds the state
  int32_t status;  // sticky error bits
  double* hist;      // optional record of (eta, a, p_a, rho) at the end of each step
  int64_t hist_cap;  // records the buffer holds
  int64_t hist_n;    // records written since the last reset
  // FP32 storage holds each field and momentum as an FP64 homogeneous offset
  // plus an FP32 remainder: phi_i = off_phi[i] + stored, pi_i = off_pi[i] +
  // stored (the pending drift applies to both parts).  FP64 storage keeps
  // the offsets at 0.  A pass forms the offsets of the state it writes,
  // off_phi + c_next off_pi and off_pi - beta dV(that), and its first tile
  // records them for the stage update (PassParams::offs).
  double off_phi[kMaxFields];
  double off_pi[kMaxFields];
};

// Homogeneous offsets of a state (see DevScalars).
struct Offsets {
  double phi[kMaxFields];
  double pi[kMaxFields];
};

// Per-lattice constants of the scalar updates.
struct BgConsts {
  double inv_dx2;    // 1/dx^2
  double inv6VLm2;   // 1/(6 V_L m_pl^2)
  double VL;         // V_L = n^3
  double VL_rho_m;   // V_L rho_m0
  double VL_rho_r;   // V_L rho_gamma0
  double mpl2;       // m_pl^2
  double dx2;
  double L;
  int32_t expand;    // 1: self-consistent expansion, 0: static a
  int32_t split;     // 1: FP32 remainders around FP64 offsets (see DevScalars)
  int32_t nf;
  int32_t pad;
};

struct PotArgs {
  double p[kMaxFields];
};

// Discrete Laplacian of eq. (2.7): weights of the centre and of the 6 face,
// 12 edge and 8 corner neighbours.  kind 0 is the 7-point member
// (-6, 1, 0, 0) with its own pass kernel; kind 1 is any member of the cubic
// family (27-point pass).
struct Stencil {
  double c[4];
  int32_t kind;
  int32_t pad;
};

// Launch shape of the tiled passes: TX lanes in x (8 .. 64) each holding VX
// consecutive sites (tile width TX*VX), TY = floor(256/TX) rows in y (the
// last 256 - TX*TY lanes of the workgroup idle), TZ planes per z-chunk.
// Pass mode pf: the prefetch depth of the z-march (1, 2 or 3 planes), plus
// kPfNontemporal when the results are written with non-temporal stores
// (7-point pass, at most two fields, 2 or 4 sites per lane).  Depth 3 comes
// with non-temporal stores only.
constexpr int kPfNontemporal = 4;
inline int pf_depth(int pf) { return pf & 3; }
inline bool pf_nt(int pf) { return (pf & kPfNontemporal) != 0; }
inline bool pf_valid(int pf) {
  return pf >= 1 && pf <= 7 && pf_depth(pf) != 0 && (pf_depth(pf) != 3 || pf_nt(pf));
}

struct Tile {
  int tx, ty, tz, vx;
  int pf;  // pass mode: prefetch depth (1, 2 or 3) | kPfNontemporal
  int ntx, nty, ntz;
  int nblocks() const { return ntx * nty * ntz; }
};

// Kernel-side view of one lattice for the fused pass.
struct PassParams {
  const void* phi[2];
  const void* pi[2];
  void* phi_w[2];
  void* pi_w[2];
  // two buffers each of the scalars, the per-tile partial sums and the
  // offset records (FP32 storage: offsets of the written state, phi[nf] then
  // pi[nf]); buffer 0 is the lattice's own, buffer 1 serves chained passes
  DevScalars* sc[2];
  double* partials[2];
  double* offs[2];
  void* sink;  // per-thread slots that absorb the stores of idle lanes
  PotArgs prm;
  BgConsts bg;
  int ntiles;  // tiles of the lattice (partials to reduce when chaining)
  double stc[4];  // stencil weights (27-point pass only)
  int n;
  int tx, ty, tz;  // lanes in x, rows, planes per chunk
  int ntx, nty, ntz;
  int zs;  // plane stride of the field arrays, in planes (LatView::zs)
};

// How one pass launch follows the previous one.  chain = 0: the scalars in
// buffer s_in are this stage's (a stage finalize or the begin kernel set
// them).  chain = 1: the pass first finishes the previous stage itself,
// exactly as the stage finalize does -- every workgroup reduces the
// previous pass's partials (buffer p_in) and advances the scalars of buffer
// s_in through that stage's end and this stage's begin -- and the first tile
// stores the result in buffer s_out for the next launch.  The pass writes
// its partials and offset record to buffer p_out.
struct Chain {
  int chain;
  int s_in, s_out, p_in, p_out;
  int eos;           // the previous stage ended a step (eta += h)
  double w_prev, w;  // weights of the previous stage and of this one
  double h;          // step size
};

// Passes chain only for lattices with at most this many tiles: every
// workgroup of a chained pass reads all partials of the previous one.
constexpr int kChainMaxTiles = 1024;

// One run of a batch for the finalize / begin kernels.
struct BatchRun {
  DevScalars* sc[2];
  double* partials[2];
  const double* offs[2];
  BgConsts bg;
  int ntiles;
  int pad;
};

// Device view of one lattice handed to the launchers.
struct LatView {
  void* phi[2];          // ping-pong field buffers, nf * n^3 each
  void* pi[2];           // ping-pong momentum buffers
  DevScalars* sc;
  double* partials;      // per-block (sum, compensation) pairs
  double* offs;          // 2 kMaxFields doubles: offsets the last pass wrote around
  // second buffers of the scalars, partials (kChainMaxTiles tiles) and
  // offset record, used by chained passes (see Chain)
  DevScalars* sc1;
  double* partials1;
  double* offs1;
  void* sink;            // kSinkBytes of store slots for idle lanes of the pass
  int n, nf, prec, pot;  // prec: sl_precision, pot: sl_potential
  // Field layout: element (field i, plane z, in-plane r = y n + x) of a phi or
  // pi array is at (z zs + i) n^2 + r.  zs = nf: the fields of a plane one
  // after the other; zs = 2 nf: phi and pi of one parity share a block, the
  // pi planes of z following its phi planes (pi[k] = phi[k] + nf n^2).
  int zs;
  PotArgs prm;
  BgConsts bg;
  Tile tile;
  Stencil st;
};

// ---- step kernels (kernels_step.hip) --------------------------------------
hipError_t launch_pass(const LatView& v, const Chain& c, hipStream_t s);
// Resident workgroups per CU of the pass kernel for this shape and stencil
// kind (the 27-point pass takes vx = 1, pf = 1 only).
int pass_blocks_per_cu(int prec, int pot, int nf, const Tile& t, int stencil_kind);
PassParams pass_params(const LatView& v);
size_t pass_lds_bytes(int prec, int nf, const Tile& t);
// Batched form: one fused pass over the tiles of nruns lattices (run table
// and tile starts in device memory), then one finalize workgroup per run.
hipError_t launch_batched_pass(int prec, int pot, int nf, const Tile& shape, int stencil_kind,
                               size_t lds, const PassParams* runs_dev, const int* start_dev,
                               int nruns, int grid, const Chain& c, hipStream_t s);
int batched_blocks_per_cu(int prec, int pot, int nf, const Tile& shape, int stencil_kind,
                          size_t lds);
// The finalize reads scalar buffer s_in and partial / offset buffer p_in and
// writes the lattice's own scalars (buffer 0).
hipError_t launch_batched_finalize(const BatchRun* runs_dev, int nruns, int s_in, int p_in,
                                   double w, double w_next, double h, int has_next,
                                   int end_of_step, hipStream_t s);
hipError_t launch_batched_begin(const BatchRun* runs_dev, int nruns, double w, double h,
                                hipStream_t s);
// Reduce the pass partials, finish stage (weight w) and, if has_next, begin
// the next stage (weight w_next); eta += h when end_of_step.
// s_in / p_in pick the scalar and partial buffers the finalize reads (0:
// the lattice's own, 1: the chaining buffers); it writes the own scalars.
hipError_t launch_stage_finalize(const LatView& v, int s_in, int p_in, double w, double w_next,
                                 double h, int has_next, int end_of_step, hipStream_t s);
// Begin the first stage of an evolve call (pending drift + H1/H2 halves).
hipError_t launch_begin(const LatView& v, double w, double h, hipStream_t s);

// ---- diagnostics (kernels_diag.hip) ---------------------------------------
// Sums at the synchronised state (per field: sum pi^2, sum G, sum (phi - s),
// sum (phi - s)^2, sum phi D phi; then sum V) into sums_dev and the
// observables into out_dev (device memory).  mode 0: observables only;
// mode 1: also set p_a from the constraint H = 0 (expanding branch) and S2.
hipError_t launch_energies(const LatView& v, double* sums_dev, sl_energies_t* out_dev, int mode,
                           hipStream_t s);
// S2 = sum pi^2 of the stored momenta into DevScalars.
hipError_t launch_sum_pi2(const LatView& v, hipStream_t s);
// phi_sync (FP64) and pi (FP64) of the current state into device staging
// buffers (either may be null).
hipError_t launch_export(const LatView& v, double* phi_out, double* pi_out, hipStream_t s);
// Store FP64 staging arrays into buffer 0 in the storage precision and reset
// the scalars: parity 0, no pending drift, eta = 0, the given a and p_a.
// off: the offsets the state is stored around (all 0 in FP64 storage).
hipError_t launch_import(const LatView& v, const double* phi_in, const double* pi_in, double a,
                         double p_a, const Offsets& off, hipStream_t s);
hipError_t launch_reset_scalars(const LatView& v, double a, double p_a, const Offsets& off,
                                hipStream_t s);
// Copy the scalars of the nruns runs of a batch table into out_dev[0 .. nruns).
hipError_t launch_gather_scalars(const BatchRun* runs_dev, int nruns, DevScalars* out_dev,
                                 hipStream_t s);

// ---- initial state and spectrum (kernels_init.hip) ------------------------
// Every site of buffer 0 = (phi0, pi0) less the state's offsets (the
// remainders are 0 in FP32 storage with offsets phi0, pi0).
hipError_t launch_fill_homogeneous(const LatView& v, const double* phi0, const double* pi0,
                                   const Offsets& off, hipStream_t s);
// Vacuum k-space amplitudes of one field into cbuf (complex FP64, n^3).
hipError_t launch_vacuum_modes(const LatView& v, double2* cbuf, int field, double m2eff,
                               double amp, uint64_t seed, hipStream_t s);
// Twiddle table tw[m] = exp(sign 2 pi i m / n).
hipError_t launch_twiddles(int n, int sign, double2* tw, hipStream_t s);
// One 1-D DFT pass along axis (0 = x, 1 = y, 2 = z) with twiddle table tw.
hipError_t launch_dft_axis(int n, const double2* in, double2* out, const double2* tw, int axis,
                           hipStream_t s);
// phi_field (buffer 0) = base + scale * Re(cbuf), rounded to storage precision.
hipError_t launch_add_real(const LatView& v, const double2* cbuf, int field, double base,
                           double scale, hipStream_t s);
// White noise of one field: phi_field (buffer 0) = base + amp (g - mean g).
hipError_t launch_white(const LatView& v, double* gbuf, double* mean_dev, int field, double base,
                        double amp, uint64_t seed, hipStream_t s);
// phi_sync of one field as the real part of cbuf.
hipError_t launch_field_to_complex(const LatView& v, int field, double2* cbuf, hipStream_t s);
// Workgroups used by the spectrum binning for side n.
int spectrum_blocks(int n);
// Shell sums of |F|^2 / n^6 of the transformed field; out3 = [k | P | count].
hipError_t launch_spectrum_bins(int n, double L, const double2* cbuf, int nbins, double* part,
                                double* out3, hipStream_t s);

// ---- energy / number spectra (spectra.hip) ---------------------------------
// m_eff^2 = lattice mean of d^2V/dphi_i^2 at the synchronised fields, per
// field, into m2_dev (part: meff_partial_doubles(nf) doubles of scratch).
size_t meff_partial_doubles(int nf);
hipError_t launch_meff(const LatView& v, double* part, double* m2_dev, hipStream_t s);
// The stored momenta of one field as the real part of cbuf.
hipError_t launch_momentum_to_complex(const LatView& v, int field, double2* cbuf, hipStream_t s);
// Binned field, energy and number spectra from the transforms F (field) and
// P (momentum) of one field; out5 = [k | <|F|^2> | <rho> | <n> | count].
int mode_spectra_blocks(int n);
hipError_t launch_mode_spectra(const LatView& v, int field, const double2* F, const double2* P,
                               int nbins, double* part, const double* m2_dev, double* out5,
                               hipStream_t s);

}  // namespace symlat
