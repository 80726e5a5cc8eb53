// Host runtime behind the C ABI of include/symlat.h: lattice handles, the
// composition driver, argument validation, the stability pre-check and the
// host<->device exchange.  Every lattice computation runs in the device
// kernels; the host only validates, allocates, launches and copies.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "timing.h"

using namespace symlat;

namespace symlat {

thread_local std::string g_last_error;

sl_status fail(sl_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

// ---------------------------------------------------------------------------
// Composition weights (Sec. 2.3): second-order map (order 2), triple jump
// eq. (2.43)-(2.44) (order 4), symmetric compositions of Table 1 (6, 8).
// ---------------------------------------------------------------------------
const double kTable1Order6[3] = {0.78451361047755726382, 0.23557321335935813368,
                                 -1.17767998417887100695};
const double kTable1Order8[7] = {0.74167036435061295345,  -0.40910082580003159400,
                                 0.19075471029623837995,  -0.57386247111608226666,
                                 0.29906418130365592384,  0.33462491824529818378,
                                 0.31529309239676659663};

std::vector<double> weights_for(int order) {
  std::vector<double> w;
  if (order == 2) {
    w = {1.0};
  } else if (order == 4) {
    const double c = std::cbrt(2.0);
    w = {1.0 / (2.0 - c), -c / (2.0 - c), 1.0 / (2.0 - c)};
  } else if (order == 6 || order == 8) {
    const double* t = order == 6 ? kTable1Order6 : kTable1Order8;
    const int half = order == 6 ? 3 : 7;
    double sum = 0.0;
    for (int i = 0; i < half; ++i) sum += t[i];
    for (int i = 0; i < half; ++i) w.push_back(t[i]);
    w.push_back(1.0 - 2.0 * sum);
    for (int i = half - 1; i >= 0; --i) w.push_back(t[i]);
  }
  return w;
}

// Largest stable omega*h of the composition on a harmonic mode (scanned at
// 1e-4 resolution and rounded down).
double stability_limit_for(int order) {
  switch (order) {
    case 2: return 2.0;
    case 4: return 1.5734;
    case 6: return 2.2690;
    case 8: return 3.3932;
    default: return -1.0;
  }
}

// d^2 V / d phi_i^2 at a homogeneous point; false where undefined.
bool hessian_diag(int kind, int nf, const double* p, const double* f, double* out) {
  switch (kind) {
    case SL_POT_FREE:
      for (int i = 0; i < nf; ++i) out[i] = p[i];
      return true;
    case SL_POT_CHAOTIC2:
      out[0] = p[0] + p[1] * f[1] * f[1];
      out[1] = p[1] * f[0] * f[0];
      return true;
    case SL_POT_OSCILLON:
      out[0] = p[0] - 3.0 * p[1] * f[0] * f[0] + 5.0 * p[2] * f[0] * f[0] * f[0] * f[0];
      return true;
    case SL_POT_QBALL_LOG: {
      const double u = 0.5 * (f[0] * f[0] + f[1] * f[1]);
      if (!(u > 0.0)) return false;
      const double base = p[0] * (1.0 + p[1] + p[1] * std::log(u / p[2]));
      out[0] = base + p[0] * p[1] * f[0] * f[0] / u;
      out[1] = base + p[0] * p[1] * f[1] * f[1] / u;
      return true;
    }
    default: return false;
  }
}

int nparams_for(int kind, int nf) {
  switch (kind) {
    case SL_POT_FREE: return nf;
    case SL_POT_CHAOTIC2: return 2;
    case SL_POT_OSCILLON: return 3;
    case SL_POT_QBALL_LOG: return 3;
    default: return -1;
  }
}

int nfields_for(int kind) {
  switch (kind) {
    case SL_POT_CHAOTIC2: return 2;
    case SL_POT_OSCILLON: return 1;
    case SL_POT_QBALL_LOG: return 2;
    default: return 0;  // any
  }
}

bool config_ok(const sl_config* c, std::string* why) {
  if (!c) { *why = "config is NULL"; return false; }
  if (c->n < 4 || c->n > 1024) { *why = "n must be in [4, 1024]"; return false; }
  if (c->nfields < 1 || c->nfields > kMaxFields) { *why = "nfields must be in [1, 8]"; return false; }
  if (!(c->L > 0.0) || !std::isfinite(c->L)) { *why = "L must be finite and > 0"; return false; }
  if (c->precision != SL_FP64 && c->precision != SL_FP32) { *why = "unknown precision"; return false; }
  if (c->expansion != SL_EXPAND_NONE && c->expansion != SL_EXPAND_SELF) {
    *why = "unknown expansion mode";
    return false;
  }
  if (!(c->mpl > 0.0) || !std::isfinite(c->mpl)) { *why = "mpl must be finite and > 0"; return false; }
  if (!(c->a0 > 0.0) || !std::isfinite(c->a0)) { *why = "a0 must be finite and > 0"; return false; }
  if (!std::isfinite(c->rho_rad0) || !std::isfinite(c->rho_mat0) || c->rho_rad0 < 0 ||
      c->rho_mat0 < 0) {
    *why = "rho_rad0 and rho_mat0 must be finite and >= 0";
    return false;
  }
  return true;
}

}  // namespace symlat

namespace {

constexpr long kMaxPassBlocks = 65536;  // bound of the per-block partial-sum buffer
constexpr int64_t kEvolveChunk = 32;     // steps per captured evolve graph
constexpr int64_t kBatchChunk = 8;       // steps per captured batch graph

// Tile geometry for lanes tx (8 .. 64), vx sites per lane, tz planes and
// prefetch depth pf.
Tile tile_geometry(int n, int tx, int vx, int tz, int pf) {
  Tile t;
  t.tx = tx;
  t.vx = vx;
  t.pf = pf;
  t.ty = kBlock / tx;
  t.ntx = (n + tx * vx - 1) / (tx * vx);
  t.nty = (n + t.ty - 1) / t.ty;
  t.tz = tz > n ? n : tz;
  t.ntz = (n + t.tz - 1) / t.tz;
  return t;
}

// Lane counts along x the tuners try for vx sites per lane: powers of two
// (8 only with 4 sites per lane, and none far wider than the lattice) and,
// when it is not one of them, the width of a whole row, so that sizes such
// as 96 run without idle columns.
std::vector<int> tx_candidates(int n, int vx) {
  std::vector<int> v;
  for (int tx : {8, 16, 32, 64}) {
    if (tx == 8 && vx != 4) continue;
    if (tx * vx > 2 * n && tx > 16) continue;
    v.push_back(tx);
  }
  const int row = n / vx;
  if (row >= 8 && row <= 64 && (row & (row - 1)) != 0) v.push_back(row);
  return v;
}

// z-chunk length for a shape: the grid should fill the resident capacity
// (blocks_per_cu * cus) in as few full rounds as possible, since a partial
// last round leaves most CUs idle; cost = rounds * (chunk + 2 halo planes).
int pick_tz(int n, int nxy, long resident) {
  double best = 1e300;
  int best_len = n;
  for (int nz = 1; nz <= n; ++nz) {
    const int len = (n + nz - 1) / nz;
    const long z = (n + len - 1) / len;
    const long blocks = long(nxy) * z;
    if (blocks > kMaxPassBlocks) break;
    const long rounds = (blocks + resident - 1) / resident;
    double est = double(rounds) * (len + 2.0);
    if (blocks * 2 < resident) est *= double(resident) / double(2 * blocks);  // too few waves
    if (est < best - 1e-9) {
      best = est;
      best_len = len;
    }
  }
  return best_len;
}

// Default lanes / sites-per-lane / prefetch depth for side n.
void default_shape(int n, int prec, int nf, int* tx, int* vx, int* pf) {
  *vx = (nf <= 2 && n % 2 == 0 && n >= 32) ? 2 : 1;
  *pf = nf <= 2 ? 2 : 1;
  (void)prec;
  const int width = n / *vx;
  *tx = width >= 64 ? 64 : (width >= 32 ? 32 : 16);
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

size_t partial_doubles() {
  const size_t pass = size_t(kMaxPassBlocks) * 6;
  const size_t diag = size_t(4096) * 2 * (5 * kMaxFields + 1);
  return pass > diag ? pass : diag;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// A lattice's device memory is two allocations: the four field arrays (each
// starting on a 256-byte boundary) and the small buffers below, at these
// offsets inside one block.
struct AuxLayout {
  size_t sc, offs, partials, sc1, offs1, partials1, sink, sums, energies, spec, total;
  AuxLayout() {
    size_t o = 0;
    auto take = [&o](size_t bytes) {
      const size_t at = o;
      o += round256(bytes);
      return at;
    };
    sc = take(sizeof(DevScalars));
    offs = take(sizeof(double) * 2 * kMaxFields);
    partials = take(partial_doubles() * sizeof(double));
    // second buffers for chained passes (lattices of at most kChainMaxTiles tiles)
    sc1 = take(sizeof(DevScalars));
    offs1 = take(sizeof(double) * 2 * kMaxFields);
    partials1 = take(size_t(kChainMaxTiles) * 6 * sizeof(double));
    sink = take(kSinkBytes);
    sums = take(sizeof(double) * (5 * kMaxFields + 1));
    energies = take(sizeof(sl_energies_t));
    spec = take(sizeof(double) * 3 * kMaxBins);
    total = o;
  }
};

// Process-wide caches of tuned pass shapes, shared by every thread of the
// process: one mutex each, lookups copy the value out.
struct TuneVal {
  int tx, vx, tz, pf;
};
template <typename K>
class ShapeCache {
 public:
  bool find(const K& k, TuneVal* v) {
    std::lock_guard<std::mutex> g(m_);
    for (const auto& kv : c_)
      if (kv.first == k) {
        *v = kv.second;
        return true;
      }
    return false;
  }
  void put(const K& k, const TuneVal& v) {
    std::lock_guard<std::mutex> g(m_);
    for (auto& kv : c_)
      if (kv.first == k) {
        kv.second = v;
        return;
      }
    c_.push_back({k, v});
  }
  void clear() {
    std::lock_guard<std::mutex> g(m_);
    c_.clear();
  }

 private:
  std::mutex m_;
  std::vector<std::pair<K, TuneVal>> c_;
};

// Autotuned single-lattice shapes keyed by (device, n, fields, precision,
// potential family, stencil kind).
struct TuneKey {
  int dev, n, nf, prec, pot, st;
  bool operator==(const TuneKey& o) const {
    return dev == o.dev && n == o.n && nf == o.nf && prec == o.prec && pot == o.pot && st == o.st;
  }
};
ShapeCache<TuneKey>& tune_cache() {
  static ShapeCache<TuneKey> c;
  return c;
}

// Process-wide cache of batch-tuned member shapes: (device, n, fields,
// precision, potential, stencil kind) plus the batch's vx and pf -> (tx, tz).
struct BatchTuneKey {
  TuneKey k;
  int vx, pf;
  bool operator==(const BatchTuneKey& o) const { return k == o.k && vx == o.vx && pf == o.pf; }
};
ShapeCache<BatchTuneKey>& batch_tune_cache() {
  static ShapeCache<BatchTuneKey> c;
  return c;
}

}  // namespace

struct sl_lattice {
  sl_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool own_fields = true;  // false: the four field arrays belong to the caller
  int device = 0;
  LatView v{};
  size_t n3 = 0;
  size_t elem = 8;
  size_t partials_n = 0;
  bool pot_set = false;
  bool state_set = false;
  int pot_kind = -1;
  double pot_raw[kMaxFields] = {0};
  double hom[kMaxFields] = {0};
  double m2max = 0.0;
  double keff2_max = 12.0;  // largest k_eff^2 of the stencil over the zone
  double a_host = 1.0;
  double* sums_dev = nullptr;
  sl_energies_t* energies_dev = nullptr;
  double* spec_dev = nullptr;
  double* hist_dev = nullptr;  // per-step background record (sl_set_history)
  void* fields_mem = nullptr;  // the four field arrays (when the handle owns them)
  void* aux_mem = nullptr;     // scalars, partial sums, sink, observable buffers
  bool timing = false;
  int chain_mode = -1;  // sl_set_chaining
  sl_batch* batch = nullptr;  // batch this lattice belongs to, if any
  int tz_user = 0;  // 0: z-chunk chosen from the occupancy of the pass kernel
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  // captured interior chunk of evolve (kEvolveChunk steps, every finalize
  // begins the next stage), replayed while (dt, order, launch view) match
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double g_dt = 0.0;
  int g_order = 0;
  LatView g_view{};
};

void batch_member_changed(sl_batch* B);
hipStream_t batch_stream(const sl_batch* B);

// Device scratch of sl_spectrum_noalloc, the spectrum entry point for
// callers that cannot allocate device memory: one array per GPU the library
// runs on, held until the process ends and shared by every such call on
// that GPU (calls that overlap on one GPU race on it).
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// Host bookkeeping of a scalar record read back from the device: the last
// finite a, and the sticky non-finite flag as SL_E_NONFINITE.
sl_status apply_scalars(sl_lattice* L, const DevScalars& S) {
  if (std::isfinite(S.a)) L->a_host = S.a;
  if (S.status & kStatusNonFinite)
    return fail(SL_E_NONFINITE, "a lattice sum or the background became non-finite");
  return SL_OK;
}

sl_status read_scalars(sl_lattice* L, DevScalars* S) {
  HIP_TRY(hipMemcpyAsync(S, L->v.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(hipStreamSynchronize(L->stream));
  return apply_scalars(L, *S);
}

sl_status require_state(sl_lattice* L) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (!L->pot_set) return fail(SL_E_STATE, "no potential set");
  if (!L->state_set) return fail(SL_E_STATE, "no initial state (call sl_init_fluctuations or sl_set_fields)");
  return SL_OK;
}

// Apply a pass shape; tz = 0 picks the z-chunk from the kernel's occupancy.
void retile(sl_lattice* L, int tx, int vx, int tz, int pf) {
  const int n = L->cfg.n;
  Tile t = tile_geometry(n, tx, vx, n, pf);
  if (tz <= 0) {
    const int bpc = L->pot_set ? pass_blocks_per_cu(L->cfg.precision, L->v.pot, L->cfg.nfields, t,
                                                    L->v.st.kind)
                               : 1;
    tz = pick_tz(n, t.ntx * t.nty, long(bpc) * device_cus());
  }
  L->v.tile = tile_geometry(n, tx, vx, tz, pf);
}

void refresh_m2max(sl_lattice* L) {
  double d2[kMaxFields];
  L->m2max = 0.0;
  if (hessian_diag(L->pot_kind, L->cfg.nfields, L->pot_raw, L->hom, d2)) {
    for (int i = 0; i < L->cfg.nfields; ++i)
      if (d2[i] > L->m2max) L->m2max = d2[i];
  }
}

void drop_graph(sl_lattice* L) {
  if (L->gexec) (void)hipGraphExecDestroy(L->gexec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->gexec = nullptr;
  L->graph = nullptr;
}

void free_all(sl_lattice* L) {
  drop_graph(L);
  if (L->fields_mem) (void)hipFree(L->fields_mem);
  if (L->aux_mem) (void)hipFree(L->aux_mem);
  if (L->hist_dev) (void)hipFree(L->hist_dev);
  for (auto& e : L->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
}

// Complex scratch for the transforms: two n^3 arrays and a twiddle table.
struct FftScratch {
  double2* a = nullptr;
  double2* b = nullptr;
  double2* tw = nullptr;
  ~FftScratch() {
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (tw) (void)hipFree(tw);
  }
};

sl_status fft_alloc(sl_lattice* L, FftScratch& S) {
  const size_t bytes = L->n3 * sizeof(double2);
  if (hipMalloc(&S.a, bytes) != hipSuccess || hipMalloc(&S.b, bytes) != hipSuccess ||
      hipMalloc(&S.tw, size_t(L->cfg.n) * sizeof(double2)) != hipSuccess)
    return fail(SL_E_NOMEM, "cannot allocate transform scratch (%zu bytes)", 2 * bytes);
  return SL_OK;
}

// 3-D DFT a -> b (a is clobbered); sign +1: sum f_n exp(+2 pi i n.j/N).
// 3-D DFT of a into b (a is overwritten); tw holds n twiddles.
sl_status dft3(sl_lattice* L, double2* a, double2* b, double2* tw, int sign) {
  const int n = L->cfg.n;
  HIP_TRY(launch_twiddles(n, sign, tw, L->stream));
  HIP_TRY(launch_dft_axis(n, a, b, tw, 0, L->stream));
  HIP_TRY(launch_dft_axis(n, b, a, tw, 1, L->stream));
  HIP_TRY(launch_dft_axis(n, a, b, tw, 2, L->stream));
  return SL_OK;
}

sl_status dft3(sl_lattice* L, FftScratch& S, int sign) { return dft3(L, S.a, S.b, S.tw, sign); }

size_t spectrum_part_bytes(int n, int nbins) {
  return size_t(spectrum_blocks(n)) * 3 * size_t(nbins) * sizeof(double);
}

// Scratch of one spectrum call: two transform buffers, the twiddles and the
// binning partials (256-byte aligned).
size_t spectrum_noalloc_bytes(int n, int nbins) {
  const size_t nn = size_t(n), n3 = nn * nn * nn;
  return round256(2 * n3 * sizeof(double2) + nn * sizeof(double2)) + spectrum_part_bytes(n, nbins);
}

sl_status spectrum_check(sl_lattice* L, int field, int nbins, const double* k_out,
                         const double* p_out, const int64_t* count_out) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (field < 0 || field >= L->cfg.nfields) return fail(SL_E_INVALID, "field index out of range");
  if (nbins < 1 || nbins > kMaxBins) return fail(SL_E_INVALID, "nbins must be in [1, %d]", kMaxBins);
  if (!k_out || !p_out || !count_out) return fail(SL_E_INVALID, "output array is NULL");
  return SL_OK;
}

// Field power spectrum with caller-provided device scratch: a, b (n^3
// complex each), tw (n complex), part (spectrum_part_bytes).  Allocates no
// device memory; synchronises the lattice's stream.
sl_status spectrum_run(sl_lattice* L, int field, int nbins, double2* a, double2* b, double2* tw,
                       double* part, double* k_out, double* p_out, int64_t* count_out) {
  std::vector<double> host(size_t(3) * nbins);
  hipError_t e = launch_field_to_complex(L->v, field, a, L->stream);
  if (e == hipSuccess) {
    const sl_status st = dft3(L, a, b, tw, -1);
    if (st != SL_OK) return st;
    e = launch_spectrum_bins(L->cfg.n, L->cfg.L, b, nbins, part, L->spec_dev, L->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(host.data(), L->spec_dev, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                       L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return fail(SL_E_DEVICE, "spectrum: %s", hipGetErrorString(e));
  for (int k = 0; k < nbins; ++k) {
    k_out[k] = host[k];
    p_out[k] = host[nbins + k];
    count_out[k] = int64_t(host[2 * nbins + k]);
  }
  DevScalars Sc;
  return read_scalars(L, &Sc);
}

// Address of this file's `scratch` array on each device, looked up once per
// device with that device current (the array's name is a host-side stand-in
// in host code; only the looked-up address may reach a kernel or a copy).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

sl_status noalloc_scratch(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return fail(SL_E_DEVICE, "device %d out of range", device);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr)
      return fail(SL_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[device];
  return SL_OK;
}

}  // namespace

extern "C" {

const char* sl_last_error(void) { return g_last_error.c_str(); }

int32_t sl_composition_weights(int32_t order, double* w_out, int32_t cap) {
  const std::vector<double> w = weights_for(order);
  if (w.empty() || !w_out || cap < int32_t(w.size())) return -1;
  for (size_t i = 0; i < w.size(); ++i) w_out[i] = w[i];
  return int32_t(w.size());
}

double sl_stability_limit(int32_t order) { return stability_limit_for(order); }

size_t sl_footprint_bytes(const sl_config* cfg) {
  std::string why;
  if (!config_ok(cfg, &why)) return 0;
  const size_t n3 = size_t(cfg->n) * cfg->n * cfg->n;
  const size_t elem = cfg->precision == SL_FP32 ? 4 : 8;
  return 4 * round256(n3 * cfg->nfields * elem) + AuxLayout().total;
}

size_t sl_transient_bytes(const sl_config* cfg) {
  std::string why;
  if (!config_ok(cfg, &why)) return 0;
  const size_t n = size_t(cfg->n), n3 = n * n * n, nf = size_t(cfg->nfields);
  const size_t fft = 2 * n3 * sizeof(double2) + n * sizeof(double2);
  const size_t staging = 2 * nf * n3 * sizeof(double);               // set/get fields
  const size_t white = n3 * sizeof(double) + sizeof(double);         // white initial state
  const size_t spectrum = fft + size_t(spectrum_blocks(cfg->n)) * 3 * kMaxBins * sizeof(double);
  const size_t spectra = fft + n3 * sizeof(double2) +
                         size_t(mode_spectra_blocks(cfg->n)) * 5 * kMaxBins * sizeof(double) +
                         meff_partial_doubles(cfg->nfields) * sizeof(double) +
                         (kMaxFields + 5 * kMaxBins) * sizeof(double);
  return std::max({fft, staging, white, spectrum, spectra});
}

namespace {

// A caller's field array: device memory of the current device, 16-byte
// aligned (vector loads), with `bytes` bytes inside one allocation.
sl_status check_user_array(void* p, size_t bytes, int device, const char* name) {
  if (!p) return fail(SL_E_INVALID, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return fail(SL_E_INVALID, "%s is not 16-byte aligned", name);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice ||
      attr.device != device) {
    (void)hipGetLastError();
    return fail(SL_E_INVALID, "%s is not device memory of device %d", name, device);
  }
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SL_E_INVALID, "%s: cannot find its allocation", name);
  }
  const uintptr_t b = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
  if (q < b || q - b > size || size - (q - b) < bytes)
    return fail(SL_E_INVALID, "%s holds fewer than the %zu bytes the lattice needs", name, bytes);
  return SL_OK;
}

sl_status create_impl(const sl_config* cfg, void* hip_stream, void* const* user, sl_lattice** out);

}  // namespace

sl_status sl_lattice_create(const sl_config* cfg, void* hip_stream, sl_lattice** out) {
  return create_impl(cfg, hip_stream, nullptr, out);
}

sl_status sl_lattice_create_with_buffers(const sl_config* cfg, void* hip_stream, void* phi0, void* pi0,
                                         void* phi1, void* pi1, sl_lattice** out) {
  void* const user[4] = {phi0, pi0, phi1, pi1};
  return create_impl(cfg, hip_stream, user, out);
}

}  // extern "C"

namespace {

sl_status create_impl(const sl_config* cfg, void* hip_stream, void* const* user, sl_lattice** out) {
  if (!out) return fail(SL_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!config_ok(cfg, &why)) return fail(SL_E_INVALID, "invalid config: %s", why.c_str());
  sl_lattice* L = new (std::nothrow) sl_lattice();
  if (!L) return fail(SL_E_NOMEM, "host allocation failed");
  L->cfg = *cfg;
  L->n3 = size_t(cfg->n) * cfg->n * cfg->n;
  L->elem = cfg->precision == SL_FP32 ? 4 : 8;
  if (hipGetDevice(&L->device) != hipSuccess) {
    delete L;
    return fail(SL_E_DEVICE, "no HIP device");
  }
  const size_t fbytes = L->n3 * cfg->nfields * L->elem;
  if (user) {
    static const char* names[4] = {"phi0", "pi0", "phi1", "pi1"};
    for (int k = 0; k < 4; ++k) {
      const sl_status st = check_user_array(user[k], fbytes, L->device, names[k]);
      if (st != SL_OK) {
        delete L;
        return st;
      }
      for (int j = 0; j < k; ++j) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(user[j]), b = reinterpret_cast<uintptr_t>(user[k]);
        if ((a < b ? b - a : a - b) < fbytes) {
          delete L;
          return fail(SL_E_INVALID, "%s and %s overlap", names[j], names[k]);
        }
      }
    }
    L->own_fields = false;
  }
  if (hip_stream) {
    L->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess) {
      delete L;
      return fail(SL_E_DEVICE, "cannot create a HIP stream");
    }
    L->own_stream = true;
  }
  LatView& v = L->v;
  v.n = cfg->n;
  v.nf = cfg->nfields;
  v.prec = cfg->precision;
  v.pot = -1;
  const double dx = cfg->L / cfg->n;
  const double VL = double(L->n3);
  v.bg.inv_dx2 = 1.0 / (dx * dx);
  v.bg.dx2 = dx * dx;
  v.bg.VL = VL;
  v.bg.inv6VLm2 = 1.0 / (6.0 * VL * cfg->mpl * cfg->mpl);
  v.bg.VL_rho_m = VL * cfg->rho_mat0;
  v.bg.VL_rho_r = VL * cfg->rho_rad0;
  v.bg.mpl2 = cfg->mpl * cfg->mpl;
  v.bg.L = cfg->L;
  v.bg.expand = cfg->expansion == SL_EXPAND_SELF ? 1 : 0;
  v.bg.split = cfg->precision == SL_FP32 ? 1 : 0;
  v.bg.nf = cfg->nfields;
  v.st = Stencil{{-6.0, 1.0, 0.0, 0.0}, 0, 0};
  {
    int tx, vx, pf;
    default_shape(cfg->n, cfg->precision, cfg->nfields, &tx, &vx, &pf);
    v.tile = tile_geometry(cfg->n, tx, vx, cfg->n, pf);
  }
  L->partials_n = partial_doubles();
  L->a_host = cfg->a0;

  bool ok = true;
  if (user) {
    v.phi[0] = user[0];
    v.pi[0] = user[1];
    v.phi[1] = user[2];
    v.pi[1] = user[3];
  }
  // The fields of a plane follow one another in every array (zs = nf).  With
  // FP64 storage of up to two fields, phi and pi of one parity also share a
  // block, interleaved by plane (zs = 2 nf, pi[k] = phi[k] + nf n^2): the
  // FP64 pass measured 2-3 % faster so, FP32 1 % slower.
  v.zs = cfg->nfields;
  if (!user) {
    const size_t stride = round256(fbytes);
    ok = hipMalloc(&L->fields_mem, 4 * stride) == hipSuccess;
    if (ok) {
      char* base = static_cast<char*>(L->fields_mem);
      if (cfg->precision == SL_FP64 && cfg->nfields <= 2) {
        const size_t plane = size_t(cfg->n) * cfg->n * cfg->nfields * L->elem;
        v.zs = 2 * cfg->nfields;
        v.phi[0] = base;
        v.pi[0] = base + plane;
        v.phi[1] = base + 2 * stride;
        v.pi[1] = base + 2 * stride + plane;
      } else {
        v.phi[0] = base;
        v.pi[0] = base + stride;
        v.phi[1] = base + 2 * stride;
        v.pi[1] = base + 3 * stride;
      }
    }
  }
  const AuxLayout aux;
  ok = ok && hipMalloc(&L->aux_mem, aux.total) == hipSuccess;
  if (ok) {
    char* base = static_cast<char*>(L->aux_mem);
    v.sc = reinterpret_cast<DevScalars*>(base + aux.sc);
    v.partials = reinterpret_cast<double*>(base + aux.partials);
    v.offs = reinterpret_cast<double*>(base + aux.offs);
    v.sc1 = reinterpret_cast<DevScalars*>(base + aux.sc1);
    v.offs1 = reinterpret_cast<double*>(base + aux.offs1);
    v.partials1 = reinterpret_cast<double*>(base + aux.partials1);
    v.sink = base + aux.sink;
    L->sums_dev = reinterpret_cast<double*>(base + aux.sums);
    L->energies_dev = reinterpret_cast<sl_energies_t*>(base + aux.energies);
    L->spec_dev = reinterpret_cast<double*>(base + aux.spec);
  }
  if (!ok) {
    free_all(L);
    delete L;
    return fail(SL_E_NOMEM, "device allocation of %zu bytes failed", sl_footprint_bytes(cfg));
  }
  if (L->fields_mem) {
    (void)hipMemsetAsync(L->fields_mem, 0, 4 * round256(fbytes), L->stream);
  } else {
    for (int k = 0; k < 2; ++k) {
      (void)hipMemsetAsync(v.phi[k], 0, fbytes, L->stream);
      (void)hipMemsetAsync(v.pi[k], 0, fbytes, L->stream);
    }
  }
  (void)hipMemsetAsync(v.sc, 0, sizeof(DevScalars), L->stream);
  (void)hipMemsetAsync(v.offs, 0, sizeof(double) * 2 * kMaxFields, L->stream);
  (void)hipMemsetAsync(v.sc1, 0, sizeof(DevScalars), L->stream);
  (void)hipMemsetAsync(v.offs1, 0, sizeof(double) * 2 * kMaxFields, L->stream);
  if (launch_reset_scalars(v, cfg->a0, 0.0, Offsets{}, L->stream) != hipSuccess ||
      hipStreamSynchronize(L->stream) != hipSuccess) {
    free_all(L);
    delete L;
    return fail(SL_E_DEVICE, "device initialisation failed");
  }
  *out = L;
  return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_lattice_destroy(sl_lattice* L) {
  if (!L) return SL_OK;
  if (L->batch) (void)sl_batch_remove(L->batch, L);
  (void)hipStreamSynchronize(L->stream);
  free_all(L);
  delete L;
  return SL_OK;
}

sl_status sl_set_potential(sl_lattice* L, int32_t kind, const double* params, int32_t nparams) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  const int nf = L->cfg.nfields;
  const int want = nparams_for(kind, nf);
  if (want < 0) return fail(SL_E_INVALID, "unknown potential kind %d", kind);
  const int nfk = nfields_for(kind);
  if (nfk && nfk != nf)
    return fail(SL_E_INVALID, "potential %d needs %d fields, lattice has %d", kind, nfk, nf);
  if (nparams != want) return fail(SL_E_INVALID, "potential %d needs %d parameters, got %d", kind, want, nparams);
  if (!params) return fail(SL_E_INVALID, "params is NULL");
  for (int i = 0; i < nparams; ++i)
    if (!std::isfinite(params[i])) return fail(SL_E_INVALID, "parameter %d is not finite", i);
  if (kind == SL_POT_QBALL_LOG && !(params[2] > 0.0)) return fail(SL_E_INVALID, "M^2 must be > 0");
  if (L->batch && kind != L->pot_kind)
    return fail(SL_E_STATE, "a batch member keeps its potential family (remove it from the batch first)");
  if (L->batch) HIP_TRY(hipStreamSynchronize(batch_stream(L->batch)));
  PotArgs dev{};
  for (int i = 0; i < nparams; ++i) {
    L->pot_raw[i] = params[i];
    dev.p[i] = params[i];
  }
  if (kind == SL_POT_QBALL_LOG) dev.p[2] = 1.0 / params[2];
  L->v.prm = dev;
  L->v.pot = kind;
  L->pot_kind = kind;
  L->pot_set = true;
  refresh_m2max(L);
  if (L->batch) {
    // a member keeps its tile (the batch's kernel is built for its per-lane
    // shape); the batch re-uploads its run table with the new parameters
    batch_member_changed(L->batch);
    return SL_OK;
  }
  const TuneKey key{L->device, L->cfg.n, L->cfg.nfields, L->cfg.precision, kind, L->v.st.kind};
  TuneVal tv;
  if (tune_cache().find(key, &tv)) {
    L->tz_user = tv.tz;
    retile(L, tv.tx, tv.vx, tv.tz, tv.pf);
    return SL_OK;
  }
  retile(L, L->v.tile.tx, L->v.tile.vx, L->tz_user, L->v.tile.pf);
  return SL_OK;
}

sl_status sl_init_fluctuations(sl_lattice* L, const double* phi0, const double* pi0, int32_t kind,
                               double amplitude, uint64_t seed) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (!L->pot_set) return fail(SL_E_STATE, "no potential set");
  if (!phi0 || !pi0) return fail(SL_E_INVALID, "phi0/pi0 is NULL");
  const int nf = L->cfg.nfields;
  for (int i = 0; i < nf; ++i)
    if (!std::isfinite(phi0[i]) || !std::isfinite(pi0[i]))
      return fail(SL_E_INVALID, "homogeneous values must be finite");
  if (kind != SL_FLUCT_NONE && kind != SL_FLUCT_VACUUM && kind != SL_FLUCT_WHITE)
    return fail(SL_E_INVALID, "unknown fluctuation kind %d", kind);
  if (!(amplitude >= 0.0) || !std::isfinite(amplitude))
    return fail(SL_E_INVALID, "amplitude must be finite and >= 0");
  double m2eff[kMaxFields];
  if (kind == SL_FLUCT_VACUUM && !hessian_diag(L->pot_kind, nf, L->pot_raw, phi0, m2eff))
    return fail(SL_E_INVALID, "effective mass undefined at the homogeneous point");

  // FP32 storage keeps the homogeneous values as FP64 offsets and stores
  // only the fluctuations; FP64 storage stores the whole values
  Offsets off{};
  double base[kMaxFields] = {};
  for (int i = 0; i < nf; ++i) {
    if (L->v.bg.split) {
      off.phi[i] = phi0[i];
      off.pi[i] = pi0[i];
    } else {
      base[i] = phi0[i];
    }
  }
  HIP_TRY(launch_reset_scalars(L->v, L->cfg.a0, 0.0, off, L->stream));
  HIP_TRY(launch_fill_homogeneous(L->v, phi0, pi0, off, L->stream));
  if (kind == SL_FLUCT_VACUUM) {
    FftScratch S;
    sl_status st = fft_alloc(L, S);
    if (st != SL_OK) return st;
    for (int i = 0; i < nf; ++i) {
      HIP_TRY(launch_vacuum_modes(L->v, S.a, i, m2eff[i], amplitude, seed, L->stream));
      st = dft3(L, S, +1);
      if (st != SL_OK) return st;
      HIP_TRY(launch_add_real(L->v, S.b, i, base[i], 1.0, L->stream));
    }
    HIP_TRY(hipStreamSynchronize(L->stream));
  } else if (kind == SL_FLUCT_WHITE) {
    double* g = nullptr;
    double* mean = nullptr;
    if (hipMalloc(&g, L->n3 * sizeof(double)) != hipSuccess ||
        hipMalloc(&mean, sizeof(double)) != hipSuccess) {
      if (g) (void)hipFree(g);
      return fail(SL_E_NOMEM, "cannot allocate white-noise scratch");
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < nf && e == hipSuccess; ++i)
      e = launch_white(L->v, g, mean, i, base[i], amplitude, seed, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    (void)hipFree(g);
    (void)hipFree(mean);
    if (e != hipSuccess) return fail(SL_E_DEVICE, "white-noise initialisation: %s", hipGetErrorString(e));
  }
  HIP_TRY(launch_energies(L->v, L->sums_dev, L->energies_dev, 1, L->stream));
  for (int i = 0; i < nf; ++i) L->hom[i] = phi0[i];
  refresh_m2max(L);
  DevScalars S;
  sl_status st = read_scalars(L, &S);
  if (st == SL_E_NONFINITE) return fail(SL_E_STATE, "constraint H = 0 has no real p_a for this state");
  if (st != SL_OK) return st;
  L->state_set = true;
  return SL_OK;
}

sl_status sl_set_fields(sl_lattice* L, const double* phi, const double* pi, double a, double p_a) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (!L->pot_set) return fail(SL_E_STATE, "no potential set");
  if (!phi || !pi) return fail(SL_E_INVALID, "phi/pi is NULL");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(SL_E_INVALID, "a must be finite and > 0");
  if (std::isinf(p_a)) return fail(SL_E_INVALID, "p_a must be finite or NaN");
  const size_t count = L->n3 * L->cfg.nfields;
  double* stage = nullptr;
  if (hipMalloc(&stage, 2 * count * sizeof(double)) != hipSuccess)
    return fail(SL_E_NOMEM, "cannot allocate staging buffers");
  hipError_t e = hipMemcpyAsync(stage, phi, count * sizeof(double), hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(stage + count, pi, count * sizeof(double), hipMemcpyHostToDevice, L->stream);
  const bool solve = std::isnan(p_a);
  // FP32 storage: remainders around each array's lattice mean (FP64 offsets)
  Offsets off{};
  if (L->v.bg.split) {
    for (int i = 0; i < L->cfg.nfields; ++i) {
      double sp = 0.0, sq = 0.0;
      for (size_t k = 0; k < L->n3; ++k) {
        sp += phi[i * L->n3 + k];
        sq += pi[i * L->n3 + k];
      }
      off.phi[i] = sp / double(L->n3);
      off.pi[i] = sq / double(L->n3);
    }
  }
  if (e == hipSuccess) e = launch_import(L->v, stage, stage + count, a, solve ? 0.0 : p_a, off, L->stream);
  if (e == hipSuccess) e = launch_sum_pi2(L->v, L->stream);
  if (e == hipSuccess && solve) e = launch_energies(L->v, L->sums_dev, L->energies_dev, 1, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  (void)hipFree(stage);
  if (e != hipSuccess) return fail(SL_E_DEVICE, "set_fields: %s", hipGetErrorString(e));
  for (int i = 0; i < L->cfg.nfields; ++i) L->hom[i] = phi[i * L->n3];
  refresh_m2max(L);
  DevScalars S;
  sl_status st = read_scalars(L, &S);
  if (st != SL_OK) {
    L->state_set = false;
    return st == SL_E_NONFINITE ? fail(SL_E_NONFINITE, "state is non-finite or the constraint has no real p_a")
                                : st;
  }
  L->state_set = true;
  return SL_OK;
}

namespace {
sl_status check_stable(sl_lattice* L, double dt, int order) {
  const double dx = L->cfg.L / L->cfg.n;
  const double omax = std::sqrt(L->keff2_max / (dx * dx) + L->a_host * L->a_host * L->m2max);
  const double lim = stability_limit_for(order);
  if (omax * std::fabs(dt) > lim)
    return fail(SL_E_UNSTABLE, "omega_max*|dt| = %.4f exceeds the order-%d stability limit %.4f",
                omax * std::fabs(dt), order, lim);
  return SL_OK;
}

// Whether the stage passes of this lattice chain (see Chain).
bool chain_passes(const LatView& v) { return v.tile.nblocks() <= kChainMaxTiles; }

}  // namespace

sl_status sl_evolve(sl_lattice* L, int64_t steps, double dt, int32_t order) {
  sl_status st = require_state(L);
  if (st != SL_OK) return st;
  if (steps < 0) return fail(SL_E_INVALID, "steps must be >= 0");
  if (!std::isfinite(dt)) return fail(SL_E_INVALID, "dt must be finite");
  const std::vector<double> w = weights_for(order);
  if (w.empty()) return fail(SL_E_INVALID, "order must be 2, 4, 6 or 8 (got %d)", order);
  st = check_stable(L, dt, order);
  if (st != SL_OK) return st;
  if (steps == 0) return SL_OK;
  const int s = int(w.size());
  // stage j of each step; has_next = 0 only for the last stage of the call.
  // A segment of nsteps steps is a chain of passes (see Chain): each pass
  // after the first finishes the previous stage itself, and one stage
  // finalize closes the segment; lattices of more than kChainMaxTiles
  // tiles run a stage finalize after every pass instead.
  const bool chained = L->chain_mode != 0 && chain_passes(L->v);
  auto enqueue_steps = [&](int64_t nsteps, bool last_chunk) -> sl_status {
    int64_t m = 0;  // pass index within the segment
    for (int64_t step = 0; step < nsteps; ++step) {
      for (int j = 0; j < s; ++j, ++m) {
        const bool last_stage = j == s - 1;
        const int has_next = !(last_stage && last_chunk && step == nsteps - 1);
        const double wn = last_stage ? w[0] : w[j + 1];
        Chain c{};
        if (chained && m > 0) {
          c.chain = 1;
          c.s_in = int((m - 1) & 1);  // pass m - 1 left its scalars there (pass 0 read buffer 0)
          c.s_out = int(m & 1);
          c.p_in = int((m - 1) & 1);
          c.eos = j == 0;
          c.w_prev = j == 0 ? w[s - 1] : w[j - 1];
          c.w = w[j];
          c.h = dt;
        }
        c.p_out = chained ? int(m & 1) : 0;
        if (L->timing) {
          hipEvent_t e0, e1;
          HIP_TRY(timing_event_create(&e0));
          HIP_TRY(timing_event_create(&e1));
          HIP_TRY(hipEventRecord(e0, L->stream));
          HIP_TRY(launch_pass(L->v, c, L->stream));
          HIP_TRY(hipEventRecord(e1, L->stream));
          L->events.emplace_back(e0, e1);
        } else {
          HIP_TRY(launch_pass(L->v, c, L->stream));
        }
        if (!chained)
          HIP_TRY(launch_stage_finalize(L->v, 0, 0, w[j], wn, dt, has_next, last_stage ? 1 : 0,
                                        L->stream));
      }
    }
    if (chained && m > 0) {
      // the last pass of the segment (index m - 1) used the scalars of
      // buffer 0 if it was the first, else those it stored in (m - 1) & 1
      const int last = int(m - 1);
      const int s_in = last == 0 ? 0 : (last & 1);
      HIP_TRY(launch_stage_finalize(L->v, s_in, last & 1, w[s - 1], w[0], dt,
                                    last_chunk ? 0 : 1, 1, L->stream));
    }
    return SL_OK;
  };
  HIP_TRY(launch_begin(L->v, w[0], dt, L->stream));
  // Interior chunks of kEvolveChunk steps replay one captured graph (the
  // same kernels with the same arguments as the eager launches); the last
  // 1 .. kEvolveChunk steps, whose final stage leaves its drift pending, and
  // timed calls are launched eagerly.
  const int64_t chunks = L->timing ? 0 : (steps - 1) / kEvolveChunk;
  if (chunks > 0) {
    if (!(L->gexec && L->g_dt == dt && L->g_order == order &&
          std::memcmp(&L->g_view, &L->v, sizeof(LatView)) == 0)) {
      drop_graph(L);
      HIP_TRY(hipStreamBeginCapture(L->stream, hipStreamCaptureModeThreadLocal));
      st = enqueue_steps(kEvolveChunk, false);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(L->stream, &g);
      if (st != SL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(SL_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
      L->graph = g;
      HIP_TRY(hipGraphInstantiate(&L->gexec, L->graph, nullptr, nullptr, 0));
      L->g_dt = dt;
      L->g_order = order;
      std::memcpy(&L->g_view, &L->v, sizeof(LatView));
    }
    for (int64_t c = 0; c < chunks; ++c) HIP_TRY(hipGraphLaunch(L->gexec, L->stream));
  }
  return enqueue_steps(steps - chunks * kEvolveChunk, true);
}

sl_status sl_set_history(sl_lattice* L, int64_t capacity) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (capacity < 0 || capacity > (int64_t(1) << 31)) return fail(SL_E_INVALID, "capacity must be in [0, 2^31]");
  // the lattice's stream and, if it is a batch member, the batch's stream
  HIP_TRY(hipStreamSynchronize(L->stream));
  if (L->batch) HIP_TRY(hipStreamSynchronize(batch_stream(L->batch)));
  DevScalars S;
  HIP_TRY(hipMemcpy(&S, L->v.sc, sizeof S, hipMemcpyDeviceToHost));
  if (capacity > 0 && L->hist_dev && S.hist == L->hist_dev && S.hist_cap == capacity) {
    S.hist_n = 0;  // same capacity: restart the record in the same buffer
    HIP_TRY(hipMemcpy(L->v.sc, &S, sizeof S, hipMemcpyHostToDevice));
    return SL_OK;
  }
  if (L->hist_dev) {
    (void)hipFree(L->hist_dev);
    L->hist_dev = nullptr;
  }
  if (capacity > 0 &&
      hipMalloc(reinterpret_cast<void**>(&L->hist_dev), size_t(capacity) * kHistRecord * sizeof(double)) != hipSuccess) {
    L->hist_dev = nullptr;
    capacity = 0;
    S.hist = nullptr;
    S.hist_cap = 0;
    S.hist_n = 0;
    HIP_TRY(hipMemcpy(L->v.sc, &S, sizeof S, hipMemcpyHostToDevice));
    return fail(SL_E_NOMEM, "cannot allocate the history buffer");
  }
  S.hist = L->hist_dev;
  S.hist_cap = capacity;
  S.hist_n = 0;
  HIP_TRY(hipMemcpy(L->v.sc, &S, sizeof S, hipMemcpyHostToDevice));
  return SL_OK;
}

sl_status sl_get_history(sl_lattice* L, double* eta, double* a, double* p_a, double* rho,
                         int64_t cap, int64_t* count) {
  if (!L || !count) return fail(SL_E_INVALID, "lattice handle or count is NULL");
  DevScalars S;
  sl_status st = read_scalars(L, &S);
  if (st != SL_OK) return st;
  *count = S.hist_n;
  const int64_t m = S.hist_n < cap ? S.hist_n : cap;
  if (m > 0) {
    if (!eta || !a || !p_a || !rho) return fail(SL_E_INVALID, "output array is NULL");
    std::vector<double> h(size_t(m) * kHistRecord);
    HIP_TRY(hipMemcpy(h.data(), L->hist_dev, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) {
      eta[i] = h[kHistRecord * i];
      a[i] = h[kHistRecord * i + 1];
      p_a[i] = h[kHistRecord * i + 2];
      rho[i] = h[kHistRecord * i + 3];
    }
  }
  return SL_OK;
}

sl_status sl_synchronize(sl_lattice* L) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  DevScalars S;
  return read_scalars(L, &S);
}

sl_status sl_get_background(sl_lattice* L, double* eta, double* a, double* p_a) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  DevScalars S;
  sl_status st = read_scalars(L, &S);
  if (eta) *eta = S.eta;
  if (a) *a = S.a;
  if (p_a) *p_a = S.p_a;
  return st;
}

sl_status sl_energies(sl_lattice* L, sl_energies_t* out) {
  sl_status st = require_state(L);
  if (st != SL_OK) return st;
  if (!out) return fail(SL_E_INVALID, "out is NULL");
  HIP_TRY(launch_energies(L->v, L->sums_dev, L->energies_dev, 0, L->stream));
  HIP_TRY(hipMemcpyAsync(out, L->energies_dev, sizeof(sl_energies_t), hipMemcpyDeviceToHost, L->stream));
  DevScalars S;
  return read_scalars(L, &S);
}

sl_status sl_get_fields(sl_lattice* L, double* phi_out, double* pi_out) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (!phi_out && !pi_out) return SL_OK;
  const size_t count = L->n3 * L->cfg.nfields;
  double* stage = nullptr;
  if (hipMalloc(&stage, 2 * count * sizeof(double)) != hipSuccess)
    return fail(SL_E_NOMEM, "cannot allocate staging buffers");
  hipError_t e = launch_export(L->v, phi_out ? stage : nullptr, pi_out ? stage + count : nullptr, L->stream);
  if (e == hipSuccess && phi_out)
    e = hipMemcpyAsync(phi_out, stage, count * sizeof(double), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess && pi_out)
    e = hipMemcpyAsync(pi_out, stage + count, count * sizeof(double), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  (void)hipFree(stage);
  if (e != hipSuccess) return fail(SL_E_DEVICE, "get_fields: %s", hipGetErrorString(e));
  DevScalars S;
  return read_scalars(L, &S);
}

sl_status sl_spectrum(sl_lattice* L, int32_t field, int32_t nbins, double* k_out, double* p_out,
                      int64_t* count_out) {
  sl_status st = spectrum_check(L, field, nbins, k_out, p_out, count_out);
  if (st != SL_OK) return st;
  FftScratch S;
  st = fft_alloc(L, S);
  if (st != SL_OK) return st;
  double* part = nullptr;
  if (hipMalloc(&part, spectrum_part_bytes(L->cfg.n, nbins)) != hipSuccess)
    return fail(SL_E_NOMEM, "cannot allocate spectrum partials");
  st = spectrum_run(L, field, nbins, S.a, S.b, S.tw, part, k_out, p_out, count_out);
  (void)hipFree(part);
  return st;
}

sl_status sl_spectrum_noalloc(sl_lattice* L, int32_t field, int32_t nbins, double* k_out,
                              double* p_out, int64_t* count_out) {
  sl_status st = spectrum_check(L, field, nbins, k_out, p_out, count_out);
  if (st != SL_OK) return st;
  const size_t n = size_t(L->cfg.n), n3 = n * n * n;
  const size_t need = spectrum_noalloc_bytes(L->cfg.n, nbins);
  if (need > kNoAllocScratchBytes)
    return fail(SL_E_INVALID,
                "sl_spectrum_noalloc: n = %d with %d bins needs %zu bytes of scratch, above its "
                "%zu-byte maximum (use sl_spectrum)",
                L->cfg.n, nbins, need, kNoAllocScratchBytes);
  unsigned char* base = nullptr;
  st = noalloc_scratch(L->device, &base);
  if (st != SL_OK) return st;
  // layout: transform buffers a, b (n^3 complex each), twiddles (n), then
  // the binning partials; every kernel writes its part before reading it
  double2* a = reinterpret_cast<double2*>(base);
  double2* b = a + n3;
  double2* tw = b + n3;
  double* part = reinterpret_cast<double*>(base + round256(2 * n3 * sizeof(double2) + n * sizeof(double2)));
  return spectrum_run(L, field, nbins, a, b, tw, part, k_out, p_out, count_out);
}

sl_status sl_spectra(sl_lattice* L, int32_t field, int32_t nbins, double* k_out, double* pf_out,
                     double* pe_out, double* pn_out, int64_t* count_out, double* m2eff_out) {
  sl_status st = require_state(L);
  if (st != SL_OK) return st;
  if (field < 0 || field >= L->cfg.nfields) return fail(SL_E_INVALID, "field index out of range");
  if (nbins < 1 || nbins > kMaxBins) return fail(SL_E_INVALID, "nbins must be in [1, %d]", kMaxBins);
  if (!k_out || !pf_out || !pe_out || !pn_out || !count_out)
    return fail(SL_E_INVALID, "output array is NULL");
  FftScratch S;
  st = fft_alloc(L, S);
  if (st != SL_OK) return st;
  const int nb = mode_spectra_blocks(L->cfg.n);
  const size_t mparts = meff_partial_doubles(L->cfg.nfields);
  double* part = nullptr;
  double* mpart = nullptr;
  double* m2 = nullptr;
  double* out5 = nullptr;
  double2* F = nullptr;
  auto release = [&]() {
    for (void* p : {static_cast<void*>(part), static_cast<void*>(mpart), static_cast<void*>(m2),
                    static_cast<void*>(out5), static_cast<void*>(F)})
      if (p) (void)hipFree(p);
  };
  if (hipMalloc(&part, size_t(nb) * 5 * nbins * sizeof(double)) != hipSuccess ||
      hipMalloc(&mpart, mparts * sizeof(double)) != hipSuccess ||
      hipMalloc(&m2, kMaxFields * sizeof(double)) != hipSuccess ||
      hipMalloc(&out5, size_t(5) * nbins * sizeof(double)) != hipSuccess ||
      hipMalloc(&F, L->n3 * sizeof(double2)) != hipSuccess) {
    release();
    return fail(SL_E_NOMEM, "cannot allocate spectrum scratch");
  }
  std::vector<double> host(size_t(5) * nbins);
  double m2h[kMaxFields] = {0};
  hipError_t e = launch_meff(L->v, mpart, m2, L->stream);
  if (e == hipSuccess) e = launch_field_to_complex(L->v, field, S.a, L->stream);
  if (e == hipSuccess) {
    st = dft3(L, S, -1);
    if (st != SL_OK) {
      release();
      return st;
    }
    e = hipMemcpyAsync(F, S.b, L->n3 * sizeof(double2), hipMemcpyDeviceToDevice, L->stream);
  }
  if (e == hipSuccess) e = launch_momentum_to_complex(L->v, field, S.a, L->stream);
  if (e == hipSuccess) {
    st = dft3(L, S, -1);
    if (st != SL_OK) {
      release();
      return st;
    }
    e = launch_mode_spectra(L->v, field, F, S.b, nbins, part, m2, out5, L->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(host.data(), out5, host.size() * sizeof(double), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m2h, m2, sizeof m2h, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  release();
  if (e != hipSuccess) return fail(SL_E_DEVICE, "spectra: %s", hipGetErrorString(e));
  for (int b = 0; b < nbins; ++b) {
    k_out[b] = host[b];
    pf_out[b] = host[nbins + b];
    pe_out[b] = host[2 * nbins + b];
    pn_out[b] = host[3 * nbins + b];
    count_out[b] = int64_t(host[4 * nbins + b]);
  }
  if (m2eff_out) *m2eff_out = m2h[field];
  DevScalars Sc;
  return read_scalars(L, &Sc);
}

sl_status sl_set_chaining(sl_lattice* L, int32_t mode) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (mode < -1 || mode > 1) return fail(SL_E_INVALID, "chaining mode must be -1, 0 or 1 (got %d)", mode);
  if (mode != L->chain_mode) {
    HIP_TRY(hipStreamSynchronize(L->stream));
    drop_graph(L);  // the captured chunk follows the mode
    L->chain_mode = mode;
  }
  return SL_OK;
}

sl_status sl_set_kernel_timing(sl_lattice* L, int32_t enable) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  L->timing = enable != 0;
  return SL_OK;
}

sl_status sl_kernel_timing(sl_lattice* L, int64_t* passes, double* total_ms) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  HIP_TRY(hipStreamSynchronize(L->stream));
  double total = 0.0;
  for (auto& e : L->events) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
    total += ms;
  }
  if (passes) *passes = int64_t(L->events.size());
  if (total_ms) *total_ms = total;
  for (auto& e : L->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  L->events.clear();
  return SL_OK;
}


sl_status sl_autotune(sl_lattice* L, int32_t reps, int32_t vx_only, int32_t pf_only,
                      int32_t* tx_out, int32_t* vx_out, int32_t* tz_out, int32_t* pf_out,
                      double* best_ms) {
  sl_status st = require_state(L);
  if (st != SL_OK) return st;
  if (reps < 1 || reps > 100) return fail(SL_E_INVALID, "reps must be in [1, 100]");
  if (vx_only != 0 && vx_only != 1 && vx_only != 2 && vx_only != 4)
    return fail(SL_E_INVALID, "vx_only must be 0, 1, 2 or 4");
  if (pf_only != 0 && !pf_valid(pf_only))
    return fail(SL_E_INVALID, "pf_only must be 0 or a pass mode (1, 2, 5 or 6)");
  const int n = L->cfg.n;
  // a batch member keeps its per-lane shape (the batch's kernel is built
  // for it)
  if (L->batch) {
    vx_only = L->v.tile.vx;
    pf_only = L->v.tile.pf;
  }
  // more than two fields: one site per lane, pf = 1; the 27-point pass:
  // one or two sites per lane, pf = 1, or two with non-temporal stores (5)
  const bool many = L->cfg.nfields > 2;
  const bool st27 = L->v.st.kind != 0;
  struct Cand {
    int tx, vx, tz, pf;
  };
  std::vector<Cand> cands;
  for (int vx : {1, 2, 4}) {
    if (n % vx != 0 || (many && vx != 1) || (st27 && vx > 2) || (vx_only && vx != vx_only)) continue;
    for (int tx : tx_candidates(n, vx)) {
      for (int pf : {1, 2, 1 | kPfNontemporal, 2 | kPfNontemporal, 3 | kPfNontemporal}) {
        if ((many && pf != 1) || (st27 && pf != 1 && pf != (1 | kPfNontemporal)) ||
            (pf_only && pf != pf_only))
          continue;
        if (pf_nt(pf) && vx < 2) continue;
        std::vector<int> tzs = {0};
        for (int d : {16, 8, 4, 2}) {
          const int tz = n / d;
          if (tz >= 8 && std::find(tzs.begin(), tzs.end(), tz) == tzs.end()) tzs.push_back(tz);
        }
        // lattices small enough to stay in the last-level cache are bound by
        // the latency of each workgroup's serial z-march, not by bandwidth:
        // short chunks give more, shorter marches
        if (n <= 128)
          for (int tz : {1, 2, 4})
            if (std::find(tzs.begin(), tzs.end(), tz) == tzs.end()) tzs.push_back(tz);
        for (int tz : tzs) {
          const Tile t = tile_geometry(n, tx, vx, tz > 0 ? tz : n, pf);
          if (long(t.nblocks()) > kMaxPassBlocks) continue;
          cands.push_back({tx, vx, tz, pf});
        }
      }
    }
  }
  if (cands.empty()) return fail(SL_E_INVALID, "no pass shape fits these constraints");
  HIP_TRY(hipStreamSynchronize(L->stream));
  const Tile saved = L->v.tile;
  const int saved_tz = L->tz_user;
  // Time real stages (pass + finalize) in the steady state of an evolve
  // call, each stage reading what the previous one wrote, with every
  // coefficient frozen at zero (no owed drift, zero step): the fields keep
  // their values, and the saved scalars are put back afterwards.
  DevScalars saved_sc;
  HIP_TRY(hipMemcpy(&saved_sc, L->v.sc, sizeof saved_sc, hipMemcpyDeviceToHost));
  DevScalars frozen = saved_sc;
  frozen.c_pend = 0.0;
  frozen.c_next = 0.0;
  frozen.alpha = 0.0;
  frozen.beta = 0.0;

  frozen.hist = nullptr;  // tuning stages are not recorded
  HIP_TRY(hipMemcpy(L->v.sc, &frozen, sizeof frozen, hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  HIP_TRY(timing_event_create(&e0));
  HIP_TRY(timing_event_create(&e1));
  auto stage = [&]() -> hipError_t {
    hipError_t e = launch_pass(L->v, Chain{}, L->stream);
    if (e == hipSuccess) e = launch_stage_finalize(L->v, 0, 0, 1.0, 1.0, 0.0, 1, 0, L->stream);
    return e;
  };
  // Each timing covers kTuneStages consecutive stages (a short sequence
  // after an idle stream favoured shapes that lose in a long run).  Shapes
  // under which sl_evolve chains its passes are timed as chained passes
  // (each finishing the previous frozen stage), after a plain stage that
  // leaves partials and offsets in buffer 0.
  constexpr int kTuneStages = 6;
  auto chained_run = [&](int nstages) -> hipError_t {
    Chain c{};
    c.chain = 1;
    c.w_prev = 1.0;
    c.w = 1.0;
    for (int k = 0; k < nstages; ++k) {
      c.s_in = c.p_in = k & 1;
      c.s_out = c.p_out = 1 - (k & 1);
      const hipError_t e = launch_pass(L->v, c, L->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  hipError_t err = hipSuccess;
  // `nstages` stages of candidate c (after a plain stage in its shape)
  // between events a and b, enqueued without waiting
  auto enqueue_timed = [&](const Cand& c, int nstages, hipEvent_t a, hipEvent_t b) {
    retile(L, c.tx, c.vx, c.tz, c.pf);
    const bool ch = L->chain_mode != 0 && chain_passes(L->v);
    if (err == hipSuccess) err = stage();
    if (err == hipSuccess) err = hipEventRecord(a, L->stream);
    if (err == hipSuccess) {
      if (ch)
        err = chained_run(nstages);
      else
        for (int k = 0; k < nstages && err == hipSuccess; ++k) err = stage();
    }
    if (err == hipSuccess) err = hipEventRecord(b, L->stream);
  };
  // milliseconds per stage between two recorded events
  auto per_stage = [&](hipEvent_t a, hipEvent_t b, int nstages) -> double {
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventSynchronize(b);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, a, b);
    return err == hipSuccess ? ms / nstages : 1e300;
  };
  // one timing of `nstages` stages of candidate c, per stage
  auto time_once = [&](const Cand& c, int nstages) -> double {
    enqueue_timed(c, nstages, e0, e1);
    return per_stage(e0, e1, nstages);
  };
  // A GPU that has been idle runs its first ~0.1 s of work at a higher
  // clock than it sustains, which favours latency-bound shapes: run frozen
  // stages of the current shape for at least kWarmMs before timing anything.
  constexpr double kWarmMs = 100.0;
  {
    const Cand cur{saved.tx, saved.vx, saved_tz, saved.pf};
    double warm = 0.0;
    for (int k = 0; k < 1000 && warm < kWarmMs && err == hipSuccess; ++k)
      warm += kTuneStages * time_once(cur, kTuneStages);
  }
  std::vector<std::pair<double, int>> timed;
  for (size_t i = 0; i < cands.size() && err == hipSuccess; ++i) {
    double t = 1e300;
    for (int r = 0; r < reps && err == hipSuccess; ++r) t = std::min(t, time_once(cands[i], kTuneStages));
    timed.emplace_back(t, int(i));
  }
  // The fastest few are timed again over four times as many stages, in
  // rounds that take them in rotating order, all enqueued back to back
  // behind a warm-up and read at the end: the GPU never idles between them,
  // as in a long run (timings separated by host waits let the clock recover
  // in the gaps, which favoured one-workgroup-per-CU shapes that lose by
  // 1-1.5 % in a long run).  Each keeps the mean of its rounds.
  std::sort(timed.begin(), timed.end());
  std::vector<int> top;
  for (size_t i = 0; i < timed.size() && i < 3; ++i)
    if (timed[i].first <= 1.05 * timed[0].first) top.push_back(timed[i].second);
  std::vector<double> t_top(top.size(), 1e300);
  if (top.size() == 1) t_top[0] = timed[0].first;
  if (top.size() > 1 && err == hipSuccess) {
    const int rounds = std::max(reps, 3);
    const int ns = 4 * kTuneStages;
    std::vector<hipEvent_t> ev(2 * top.size() * rounds, nullptr);
    for (size_t k = 0; k < ev.size() && err == hipSuccess; ++k) err = timing_event_create(&ev[k]);
    enqueue_timed(cands[top[0]], 8 * kTuneStages, e0, e1);
    for (int r = 0; r < rounds && err == hipSuccess; ++r)
      for (size_t j = 0; j < top.size() && err == hipSuccess; ++j) {
        const size_t i = (j + r) % top.size();
        const size_t k = 2 * (size_t(r) * top.size() + i);
        enqueue_timed(cands[top[i]], ns, ev[k], ev[k + 1]);
      }
    std::fill(t_top.begin(), t_top.end(), 0.0);
    for (int r = 0; r < rounds && err == hipSuccess; ++r)
      for (size_t i = 0; i < top.size() && err == hipSuccess; ++i) {
        const size_t k = 2 * (size_t(r) * top.size() + i);
        t_top[i] += per_stage(ev[k], ev[k + 1], ns) / rounds;
      }
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  double best = 1e300;
  Cand win = cands[0];
  for (size_t i = 0; i < top.size(); ++i)
    if (t_top[i] < best) {
      best = t_top[i];
      win = cands[top[i]];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the buffer saved_sc.parity names holds the state (a frozen stage writes
  // back the values it read)
  const hipError_t er = hipStreamSynchronize(L->stream);
  const hipError_t ec = hipMemcpy(L->v.sc, &saved_sc, sizeof saved_sc, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = er != hipSuccess ? er : ec;
  if (err != hipSuccess) {
    L->v.tile = saved;
    L->tz_user = saved_tz;
    return fail(SL_E_DEVICE, "autotune: %s", hipGetErrorString(err));
  }
  L->tz_user = win.tz;
  retile(L, win.tx, win.vx, win.tz, win.pf);
  const TuneKey key{L->device, n, L->cfg.nfields, L->cfg.precision, L->v.pot, L->v.st.kind};
  tune_cache().put(key, {win.tx, win.vx, win.tz, win.pf});
  if (L->batch) batch_member_changed(L->batch);
  if (tx_out) *tx_out = win.tx;
  if (vx_out) *vx_out = win.vx;
  if (tz_out) *tz_out = L->v.tile.tz;
  if (pf_out) *pf_out = win.pf;
  if (best_ms) *best_ms = best;
  return SL_OK;
}

sl_status sl_autotune_forget(void) {
  tune_cache().clear();
  batch_tune_cache().clear();
  return SL_OK;
}

sl_status sl_get_tile(sl_lattice* L, int32_t* tx, int32_t* vx, int32_t* ty, int32_t* tz,
                      int32_t* pf) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (tx) *tx = L->v.tile.tx;
  if (vx) *vx = L->v.tile.vx;
  if (ty) *ty = L->v.tile.ty;
  if (tz) *tz = L->v.tile.tz;
  if (pf) *pf = L->v.tile.pf;
  return SL_OK;
}

sl_status sl_set_tile(sl_lattice* L, int32_t tx, int32_t vx, int32_t tz, int32_t pf) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (tx < 8 || tx > 64) return fail(SL_E_INVALID, "tx must be in [8, 64]");
  if (vx != 1 && vx != 2 && vx != 4) return fail(SL_E_INVALID, "vx must be 1, 2 or 4");
  if (L->cfg.n % vx != 0) return fail(SL_E_INVALID, "vx = %d needs n divisible by %d", vx, vx);
  if (!pf_valid(pf)) return fail(SL_E_INVALID, "pf must be 1, 2, 5, 6 or 7 (depth 1, 2 or 3, plus 4 for non-temporal stores)");
  if (L->cfg.nfields > 2 && (vx != 1 || pf != 1))
    return fail(SL_E_INVALID, "more than two fields run with vx = 1 and pf = 1 only");
  if (L->v.st.kind != 0 && (vx > 2 || (pf != 1 && pf != (1 | kPfNontemporal))))
    return fail(SL_E_INVALID, "the 27-point stencil runs with vx = 1 or 2 and pf = 1, or vx = 2 and pf = 5");
  if (pf_nt(pf) && vx < 2) return fail(SL_E_INVALID, "non-temporal stores need vx = 2 or 4");
  if (L->batch && (vx != L->v.tile.vx || pf != L->v.tile.pf))
    return fail(SL_E_STATE, "a batch member keeps its vx and pf (remove it from the batch first)");
  if (tz < 0 || tz > L->cfg.n) return fail(SL_E_INVALID, "tz must be in [0, n]");
  const Tile t = tile_geometry(L->cfg.n, tx, vx, tz > 0 ? tz : L->cfg.n, pf);
  if (long(t.nblocks()) > kMaxPassBlocks)
    return fail(SL_E_INVALID, "tile gives %d workgroups (limit %ld)", t.nblocks(), kMaxPassBlocks);
  HIP_TRY(hipStreamSynchronize(L->stream));
  L->tz_user = tz;
  retile(L, tx, vx, tz, pf);
  if (L->batch) batch_member_changed(L->batch);
  return SL_OK;
}

sl_status sl_set_stencil(sl_lattice* L, const double* c) {
  if (!L) return fail(SL_E_INVALID, "lattice handle is NULL");
  if (!c) return fail(SL_E_INVALID, "coefficients are NULL");
  double scale = 1.0;
  for (int k = 0; k < 4; ++k) {
    if (!std::isfinite(c[k])) return fail(SL_E_INVALID, "coefficient %d is not finite", k);
    scale += std::fabs(c[k]) * (k == 0 ? 1 : (k == 1 ? 6 : (k == 2 ? 12 : 8)));
  }
  if (std::fabs(c[0] + 6.0 * c[1] + 12.0 * c[2] + 8.0 * c[3]) > 1e-12 * scale)
    return fail(SL_E_INVALID, "stencil must annihilate constants: c0 + 6 c1 + 12 c2 + 8 c3 = 0");
  if (std::fabs(c[1] + 4.0 * c[2] + 4.0 * c[3] - 1.0) > 1e-12 * scale)
    return fail(SL_E_INVALID, "stencil must tend to the Laplacian: c1 + 4 c2 + 4 c3 = 1");
  const int kind = (c[0] == -6.0 && c[1] == 1.0 && c[2] == 0.0 && c[3] == 0.0) ? 0 : 1;
  if (L->batch && kind != L->v.st.kind)
    return fail(SL_E_STATE, "a batch member keeps its stencil kind (remove it from the batch first)");
  HIP_TRY(hipStreamSynchronize(L->stream));
  Stencil st{{c[0], c[1], c[2], c[3]}, kind, 0};
  // the symbol is multilinear in the three cosines: its extremes over the
  // zone sit at the vertices k_d in {0, pi}
  double kmax = 0.0;
  for (int v = 0; v < 8; ++v) {
    const double cz = (v & 4) ? -1.0 : 1.0, cy = (v & 2) ? -1.0 : 1.0, cx = (v & 1) ? -1.0 : 1.0;
    const double sym = c[0] + 2.0 * c[1] * (cz + cy + cx) + 4.0 * c[2] * (cz * cy + cz * cx + cy * cx) +
                       8.0 * c[3] * cz * cy * cx;
    if (-sym > kmax) kmax = -sym;
  }
  const int old_kind = L->v.st.kind;
  L->v.st = st;
  L->keff2_max = kmax;
  if (kind != old_kind) {
    int tx = L->v.tile.tx, vx = L->v.tile.vx, pf = L->v.tile.pf;
    if (kind != 0) {
      vx = (L->cfg.nfields <= 2 && L->cfg.n % 2 == 0 && L->cfg.n >= 32) ? 2 : 1;
      pf = 1;
      const int width = L->cfg.n / vx;
      tx = width >= 64 ? 64 : (width >= 32 ? 32 : 16);
    } else {
      default_shape(L->cfg.n, L->cfg.precision, L->cfg.nfields, &tx, &vx, &pf);
    }
    if (L->pot_set) {
      const TuneKey key{L->device, L->cfg.n, L->cfg.nfields, L->cfg.precision, L->v.pot, kind};
      TuneVal tv;
      if (tune_cache().find(key, &tv)) {
        tx = tv.tx;
        vx = tv.vx;
        pf = tv.pf;
        L->tz_user = tv.tz;
      }
    }
    retile(L, tx, vx, L->tz_user, pf);
  }
  if (L->batch) batch_member_changed(L->batch);
  return SL_OK;
}

sl_status sl_get_stencil(sl_lattice* L, double* c_out) {
  if (!L || !c_out) return fail(SL_E_INVALID, "lattice handle or output is NULL");
  for (int k = 0; k < 4; ++k) c_out[k] = L->v.st.c[k];
  return SL_OK;
}


// ---------------------------------------------------------------------------
// Batches: many lattices (same storage precision, potential family, field
// count and per-lane shape; any sizes and parameters) advanced together.
// ---------------------------------------------------------------------------
}  // extern "C"

struct sl_batch {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<sl_lattice*> runs;
  int prec = -1, pot = -1, nf = -1;
  Tile shape{};  // carries vx and pf of every member
  int st_kind = 0;  // stencil kind of every member
  PassParams* pass_dev = nullptr;
  BatchRun* run_dev = nullptr;
  int* start_dev = nullptr;
  DevScalars* sc_dev = nullptr;        // members' scalars gathered for one read-back
  std::vector<DevScalars> sc_host;
  int cap = 0;
  bool dirty = true;
  int total_tiles = 0;
  size_t lds = 0;
  int grid_req = 0;  // 0: one workgroup per tile; > 0: that many workgroups stride through them
  int grid = 0;      // workgroups of the batched pass as last uploaded
  uint64_t version = 0;
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double g_dt = 0.0;
  int g_order = 0;
  uint64_t g_version = ~0ull;
};

namespace {

}  // namespace

// A member's tile or stencil changed: re-upload the run table and capture
// a new graph at the next step.
hipStream_t batch_stream(const sl_batch* B) { return B->stream; }

void batch_member_changed(sl_batch* B) {
  B->dirty = true;
  ++B->version;
}

namespace {

// Workgroups of the batched pass.  By default one per tile: the dispatcher
// hands the next tile to whichever CU frees a slot first, which evens out
// tiles of different sizes.  A requested count (the persistent form) makes
// each XCD's workgroups stride through its contiguous range of tiles.
int batch_grid(int requested, int total_tiles) {
  const int total = total_tiles > 0 ? total_tiles : 1;
  return requested > 0 && requested < total ? requested : total;
}

void batch_drop_graph(sl_batch* B) {
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->gexec = nullptr;
  B->graph = nullptr;
  B->g_version = ~0ull;
}

sl_status batch_upload(sl_batch* B) {
  const int R = int(B->runs.size());
  if (R > B->cap) {
    batch_drop_graph(B);
    if (B->pass_dev) (void)hipFree(B->pass_dev);
    if (B->run_dev) (void)hipFree(B->run_dev);
    if (B->start_dev) (void)hipFree(B->start_dev);
    if (B->sc_dev) (void)hipFree(B->sc_dev);
    B->pass_dev = nullptr;
    B->run_dev = nullptr;
    B->start_dev = nullptr;
    B->sc_dev = nullptr;
    int cap = B->cap ? B->cap : 16;
    while (cap < R) cap *= 2;
    if (hipMalloc(&B->pass_dev, sizeof(PassParams) * cap) != hipSuccess ||
        hipMalloc(&B->run_dev, sizeof(BatchRun) * cap) != hipSuccess ||
        hipMalloc(&B->start_dev, sizeof(int) * (cap + 1)) != hipSuccess ||
        hipMalloc(&B->sc_dev, sizeof(DevScalars) * cap) != hipSuccess) {
      B->cap = 0;
      return fail(SL_E_NOMEM, "cannot allocate the batch run table");
    }
    B->cap = cap;
  }
  std::vector<PassParams> pp(R);
  std::vector<BatchRun> br(R);
  std::vector<int> start(R + 1, 0);
  size_t lds = 0;
  for (int r = 0; r < R; ++r) {
    sl_lattice* L = B->runs[r];
    pp[r] = pass_params(L->v);
    br[r].sc[0] = L->v.sc;
    br[r].sc[1] = L->v.sc1;
    br[r].partials[0] = L->v.partials;
    br[r].partials[1] = L->v.partials1;
    br[r].offs[0] = L->v.offs;
    br[r].offs[1] = L->v.offs1;
    br[r].bg = L->v.bg;
    br[r].ntiles = L->v.tile.nblocks();
    br[r].pad = 0;
    start[r + 1] = start[r] + br[r].ntiles;
    const size_t l = pass_lds_bytes(B->prec, B->nf, L->v.tile);
    if (l > lds) lds = l;
  }
  HIP_TRY(hipMemcpyAsync(B->pass_dev, pp.data(), sizeof(PassParams) * R, hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipMemcpyAsync(B->run_dev, br.data(), sizeof(BatchRun) * R, hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipMemcpyAsync(B->start_dev, start.data(), sizeof(int) * (R + 1), hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->total_tiles = start[R];
  B->lds = lds;
  B->grid = batch_grid(B->grid_req, B->total_tiles);
  B->dirty = false;
  return SL_OK;
}

// Enqueue one batched evolve call on the batch stream.
// `steps` steps of every member; has_next = 0 only for the last stage of the
// call's last chunk, whose drift then stays pending.
sl_status batch_enqueue(sl_batch* B, int64_t steps, double dt, const std::vector<double>& w,
                        bool last_chunk) {
  // batches do not chain (see Chain): a workgroup of the batched pass may
  // run several tiles in turn, and the members' tiles are short
  const int R = int(B->runs.size());
  const int s = int(w.size());
  for (int64_t step = 0; step < steps; ++step) {
    for (int j = 0; j < s; ++j) {
      const bool last_stage = j == s - 1;
      const int has_next = !(last_stage && last_chunk && step == steps - 1);
      const double wn = last_stage ? w[0] : w[j + 1];
      HIP_TRY(launch_batched_pass(B->prec, B->pot, B->nf, B->shape, B->st_kind, B->lds, B->pass_dev,
                                  B->start_dev, R, B->grid, Chain{}, B->stream));
      HIP_TRY(launch_batched_finalize(B->run_dev, R, 0, 0, w[j], wn, dt, has_next,
                                      last_stage ? 1 : 0, B->stream));
    }
  }
  return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_batch_create(void* hip_stream, sl_batch** out) {
  if (!out) return fail(SL_E_INVALID, "out is NULL");
  *out = nullptr;
  sl_batch* B = new (std::nothrow) sl_batch();
  if (!B) return fail(SL_E_NOMEM, "host allocation failed");
  if (hip_stream) {
    B->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess) {
      delete B;
      return fail(SL_E_DEVICE, "cannot create a HIP stream");
    }
    B->own_stream = true;
  }
  if (hipEventCreateWithFlags(&B->ev, hipEventDisableTiming) != hipSuccess) {
    if (B->own_stream) (void)hipStreamDestroy(B->stream);
    delete B;
    return fail(SL_E_DEVICE, "cannot create a HIP event");
  }
  *out = B;
  return SL_OK;
}

sl_status sl_batch_destroy(sl_batch* B) {
  if (!B) return SL_OK;
  (void)hipStreamSynchronize(B->stream);
  for (sl_lattice* L : B->runs) L->batch = nullptr;
  batch_drop_graph(B);
  if (B->pass_dev) (void)hipFree(B->pass_dev);
  if (B->run_dev) (void)hipFree(B->run_dev);
  if (B->start_dev) (void)hipFree(B->start_dev);
  if (B->sc_dev) (void)hipFree(B->sc_dev);
  if (B->ev) (void)hipEventDestroy(B->ev);
  if (B->own_stream) (void)hipStreamDestroy(B->stream);
  delete B;
  return SL_OK;
}

sl_status sl_batch_add(sl_batch* B, sl_lattice* L) {
  if (!B || !L) return fail(SL_E_INVALID, "batch or lattice handle is NULL");
  sl_status st = require_state(L);
  if (st != SL_OK) return st;
  if (L->batch) return fail(SL_E_INVALID, "lattice already belongs to a batch");
  if (!B->runs.empty() &&
      (L->cfg.precision != B->prec || L->v.pot != B->pot || L->cfg.nfields != B->nf ||
       L->v.st.kind != B->st_kind))
    return fail(SL_E_INVALID,
                "batch members share precision, potential family, field count and stencil kind");
  HIP_TRY(hipStreamSynchronize(B->stream));
  // a size the batch tuner has seen starts with its tuned shape; a member
  // takes the batch's per-lane shape (vx, pf)
  int tx = L->v.tile.tx, vx = L->v.tile.vx, tz = L->tz_user, pf = L->v.tile.pf;
  const BatchTuneKey key{{L->device, L->cfg.n, L->cfg.nfields, L->cfg.precision, L->v.pot, L->v.st.kind},
                         0, 0};
  TuneVal tv;
  if (batch_tune_cache().find(key, &tv)) {
    tx = tv.tx;
    vx = tv.vx;
    tz = tv.tz;
    pf = tv.pf;
  }
  if (!B->runs.empty() && (vx != B->shape.vx || pf != B->shape.pf)) {
    vx = B->shape.vx;
    pf = B->shape.pf;
    if (L->cfg.n % vx != 0)
      return fail(SL_E_INVALID, "n = %d is not a multiple of the batch's vx = %d", L->cfg.n, vx);
    const int width = L->cfg.n / vx;
    tx = width >= 64 ? 64 : (width >= 32 ? 32 : 16);
    tz = 0;
  }
  if (tx != L->v.tile.tx || vx != L->v.tile.vx || pf != L->v.tile.pf || tz != L->tz_user) {
    HIP_TRY(hipStreamSynchronize(L->stream));
    L->tz_user = tz;
    retile(L, tx, vx, tz, pf);
  }
  if (B->runs.empty()) {
    B->prec = L->cfg.precision;
    B->pot = L->v.pot;
    B->nf = L->cfg.nfields;
    B->shape = L->v.tile;
    B->st_kind = L->v.st.kind;
  }
  B->runs.push_back(L);
  L->batch = B;
  B->dirty = true;
  ++B->version;
  return SL_OK;
}

sl_status sl_batch_remove(sl_batch* B, sl_lattice* L) {
  if (!B || !L) return fail(SL_E_INVALID, "batch or lattice handle is NULL");
  for (size_t i = 0; i < B->runs.size(); ++i) {
    if (B->runs[i] == L) {
      HIP_TRY(hipStreamSynchronize(B->stream));
      B->runs.erase(B->runs.begin() + long(i));
      L->batch = nullptr;
      B->dirty = true;
      ++B->version;
      if (B->runs.empty()) B->prec = B->pot = B->nf = -1;
      return SL_OK;
    }
  }
  return fail(SL_E_INVALID, "lattice is not in this batch");
}

}  // extern "C"

namespace {

// Consecutive batched passes per timing: short windows after a host wait
// run at a recovered clock, and their noise made the batch tuner's choice
// among near-equal shapes change from process to process.
constexpr int kBatchTimedPasses = 4;

// Time the batched pass alone with the current shapes: without its
// finalize it leaves every member's state as it was (it reads the current
// buffer and writes the spare buffer and the partials).  Best of `reps`
// timings of kBatchTimedPasses consecutive passes, per pass.

sl_status batch_time_pass(sl_batch* B, int reps, hipEvent_t e0, hipEvent_t e1, double* ms_out) {
  sl_status st = batch_upload(B);
  if (st != SL_OK) return st;
  double best = 1e300;
  HIP_TRY(launch_batched_pass(B->prec, B->pot, B->nf, B->shape, B->st_kind, B->lds, B->pass_dev,
                              B->start_dev, int(B->runs.size()), B->grid, Chain{}, B->stream));
  for (int r = 0; r < reps; ++r) {
    HIP_TRY(hipEventRecord(e0, B->stream));
    for (int k = 0; k < kBatchTimedPasses; ++k)
      HIP_TRY(launch_batched_pass(B->prec, B->pot, B->nf, B->shape, B->st_kind, B->lds, B->pass_dev,
                                  B->start_dev, int(B->runs.size()), B->grid, Chain{}, B->stream));
    HIP_TRY(hipEventRecord(e1, B->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms / kBatchTimedPasses < best) best = ms / kBatchTimedPasses;
  }
  *ms_out = best;
  return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_batch_time_pass(sl_batch* B, int32_t reps, double* ms) {
  if (!B || !ms) return fail(SL_E_INVALID, "batch handle or output is NULL");
  if (reps < 1 || reps > 100) return fail(SL_E_INVALID, "reps must be in [1, 100]");
  if (B->runs.empty()) return fail(SL_E_STATE, "the batch has no members");
  for (sl_lattice* L : B->runs) HIP_TRY(hipStreamSynchronize(L->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  hipEvent_t e0, e1;
  HIP_TRY(timing_event_create(&e0));
  HIP_TRY(timing_event_create(&e1));
  const sl_status st = batch_time_pass(B, reps, e0, e1, ms);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

sl_status sl_batch_autotune(sl_batch* B, int32_t reps, double* best_ms) {
  if (!B) return fail(SL_E_INVALID, "batch handle is NULL");
  if (reps < 1 || reps > 100) return fail(SL_E_INVALID, "reps must be in [1, 100]");
  if (B->runs.empty()) return fail(SL_E_STATE, "the batch has no members");
  for (sl_lattice* L : B->runs) HIP_TRY(hipStreamSynchronize(L->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  // member sizes, largest share of the sites first
  std::vector<std::pair<double, int>> sizes;
  for (sl_lattice* L : B->runs) {
    bool seen = false;
    for (auto& s : sizes)
      if (s.second == L->cfg.n) {
        s.first += double(L->n3);
        seen = true;
      }
    if (!seen) sizes.push_back({double(L->n3), L->cfg.n});
  }
  std::sort(sizes.begin(), sizes.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first > b.first;
  });
  hipEvent_t e0, e1;
  HIP_TRY(timing_event_create(&e0));
  HIP_TRY(timing_event_create(&e1));
  auto time_now = [&](double* ms_out) -> sl_status {
    return batch_time_pass(B, reps, e0, e1, ms_out);
  };
  auto apply = [&](int n, int tx, int vx, int tz, int pf) {
    for (sl_lattice* L : B->runs)
      if (L->cfg.n == n) {
        L->tz_user = tz;
        retile(L, tx, vx, tz, pf);
      }
    B->shape.vx = vx;
    B->shape.pf = pf;
    B->dirty = true;
  };
  auto cur_shape = [&](int n, int* tx, int* tz) {
    for (sl_lattice* L : B->runs)
      if (L->cfg.n == n) {
        *tx = L->v.tile.tx;
        *tz = L->v.tile.tz;
      }
  };
  // per-lane shapes every member can take
  std::vector<std::pair<int, int>> lane_shapes;
  for (int vx : {1, 2, 4}) {
    bool ok = !(B->nf > 2 && vx != 1) && !(B->st_kind != 0 && vx > 2);
    for (const auto& sz : sizes) ok = ok && sz.second % vx == 0;
    for (int pf : {1, 2, 1 | kPfNontemporal, 2 | kPfNontemporal, 3 | kPfNontemporal})
      if (ok && !(B->nf > 2 && pf != 1) && !(B->st_kind != 0 && pf != 1 && pf != (1 | kPfNontemporal)) &&
          !(pf_nt(pf) && vx < 2))
        lane_shapes.push_back({vx, pf});
  }
  batch_drop_graph(B);
  // shapes are tuned with one workgroup per tile; phase 3 picks the grid
  const int saved_grid = B->grid_req;
  B->grid_req = 0;
  B->dirty = true;
  struct Pick {
    int tx, tz;
  };
  std::vector<Pick> best_pick(sizes.size());
  int best_vx = B->shape.vx, best_pf = B->shape.pf;
  double best_all = 1e300;
  sl_status st = SL_OK;
  // set every size to a lane shape: the members' current shapes for the
  // batch's own lane shape, else a whole row per tile (at most 64 lanes, at
  // least 8) with a quarter-lattice chunk
  auto start_shape = [&](int vx, int pf) {
    for (const auto& sz : sizes) {
      const int n = sz.second;
      int tx = 0, tz = 0;
      cur_shape(n, &tx, &tz);
      if (vx != B->shape.vx || pf != B->shape.pf) {
        const int width = n / vx;
        tx = width > 64 ? 64 : (width < 8 ? 8 : width);
        tz = n / 4 >= 4 ? n / 4 : n;
      }
      apply(n, tx, vx, tz, pf);
    }
  };
  // phase 1: every lane shape at its starting shapes; phase 2 refines the
  // three best.  A shape (or lane shape) replaces the current one only when
  // it is faster by more than the timing noise (kBatchGain), twice: once in
  // the scan and again when the two are timed one right after the other,
  // so that the choice is the same from process to process.
  constexpr double kBatchGain = 0.99;
  const int orig_vx = B->shape.vx, orig_pf = B->shape.pf;
  // An idle GPU runs its first ~0.1 s of work at a higher clock than it
  // sustains, which favoured the lane shapes timed first: run the current
  // shapes for at least that long before timing anything.
  {
    double warm = 0.0;
    for (int k = 0; k < 1000 && warm < 100.0 && st == SL_OK; ++k) {
      double ms = 0.0;
      st = time_now(&ms);
      warm += ms * (1 + kBatchTimedPasses * reps);
    }
  }
  std::vector<std::pair<double, int>> ranked;
  for (size_t q = 0; q < lane_shapes.size() && st == SL_OK; ++q) {
    B->shape.vx = orig_vx;
    B->shape.pf = orig_pf;
    start_shape(lane_shapes[q].first, lane_shapes[q].second);
    double ms = 0.0;
    st = time_now(&ms);
    ranked.push_back({ms, int(q)});
  }
  std::sort(ranked.begin(), ranked.end());
  for (size_t r = 0; r < ranked.size() && r < 3 && st == SL_OK; ++r) {
    const int vx = lane_shapes[ranked[r].second].first, pf = lane_shapes[ranked[r].second].second;
    B->shape.vx = orig_vx;
    B->shape.pf = orig_pf;
    start_shape(vx, pf);
    double cur = 0.0;
    st = time_now(&cur);
    for (int round = 0; round < 2 && st == SL_OK; ++round) {
      for (const auto& sz : sizes) {
        const int n = sz.second;
        int ref_tx = 0, ref_tz = 0;
        cur_shape(n, &ref_tx, &ref_tz);
        int btx = ref_tx, btz = ref_tz;
        for (int tx : tx_candidates(n, vx)) {
          if (B->st_kind != 0 && 2 * tx + 2 * (kBlock / tx) + 4 > kBlock) continue;
          for (int d : {1, 2, 3, 4, 6, 8}) {
            if (d % 3 == 0 && n % d != 0) continue;  // thirds only where they divide n
            const int tz = n / d;
            if (tz < 4 && d != 1) continue;
            if (tx == ref_tx && tz == ref_tz) continue;
            const Tile t = tile_geometry(n, tx, vx, tz, pf);
            if (long(t.nblocks()) > kMaxPassBlocks) continue;
            apply(n, tx, vx, tz, pf);
            double ms = 0.0;
            st = time_now(&ms);
            if (st != SL_OK) break;
            if (ms < cur * kBatchGain) {
              // confirm: the current shape and the candidate timed again,
              // one right after the other
              double ms_ref = 0.0, ms_new = 0.0;
              apply(n, btx, vx, btz, pf);
              st = time_now(&ms_ref);
              if (st == SL_OK) {
                apply(n, tx, vx, tz, pf);
                st = time_now(&ms_new);
              }
              if (st != SL_OK) break;
              if (ms_new < ms_ref * kBatchGain) {
                cur = ms_new;
                btx = tx;
                btz = tz;
              } else {
                cur = ms_ref;
              }
            }
          }
          if (st != SL_OK) break;
        }
        apply(n, btx, vx, btz, pf);
        if (st != SL_OK) break;
      }
    }
    if (st != SL_OK) break;
    if (cur < best_all * kBatchGain && best_all < 1e299) {
      // confirm against the best lane shape so far, both timed again
      std::vector<Pick> mine(sizes.size());
      for (size_t i = 0; i < sizes.size(); ++i) cur_shape(sizes[i].second, &mine[i].tx, &mine[i].tz);
      double ms_ref = 0.0, ms_new = 0.0;
      for (size_t i = 0; i < sizes.size(); ++i)
        apply(sizes[i].second, best_pick[i].tx, best_vx, best_pick[i].tz, best_pf);
      st = time_now(&ms_ref);
      for (size_t i = 0; i < sizes.size(); ++i) apply(sizes[i].second, mine[i].tx, vx, mine[i].tz, pf);
      if (st == SL_OK) st = time_now(&ms_new);
      if (st != SL_OK) break;
      if (ms_new < ms_ref * kBatchGain) {
        cur = ms_new;
      } else {
        best_all = ms_ref;
        cur = 1e300;  // keep the earlier lane shape
      }
    }
    if (cur < best_all * kBatchGain) {
      best_all = cur;
      best_vx = vx;
      best_pf = pf;
      for (size_t i = 0; i < sizes.size(); ++i) cur_shape(sizes[i].second, &best_pick[i].tx, &best_pick[i].tz);
    }
  }
  if (st == SL_OK) {
    for (size_t i = 0; i < sizes.size(); ++i)
      apply(sizes[i].second, best_pick[i].tx, best_vx, best_pick[i].tz, best_pf);
    // phase 3: one workgroup per tile against the persistent form with a
    // grid of the resident capacity; the persistent form only if 0.5 %
    // faster
    double t_tile = 0.0, t_pers = 0.0;
    st = time_now(&t_tile);
    const long resident = long(batched_blocks_per_cu(B->prec, B->pot, B->nf, B->shape, B->st_kind,
                                                     B->lds)) * device_cus();
    if (st == SL_OK && resident < B->total_tiles) {
      B->grid_req = int(resident);
      B->dirty = true;
      st = time_now(&t_pers);
    }
    if (st == SL_OK) {
      if (t_pers > 0.0 && t_pers < 0.995 * t_tile) {
        best_all = t_pers;
      } else {
        B->grid_req = 0;
        best_all = t_tile;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SL_OK) {
    B->grid_req = saved_grid;
    B->dirty = true;
    ++B->version;
    return st;
  }
  // remember the shapes for members added later (this batch or another)
  for (size_t i = 0; i < sizes.size(); ++i) {
    const sl_lattice* R = nullptr;
    for (sl_lattice* L : B->runs)
      if (L->cfg.n == sizes[i].second) R = L;
    const BatchTuneKey key{{R->device, R->cfg.n, R->cfg.nfields, R->cfg.precision, R->v.pot, R->v.st.kind},
                           0, 0};
    const TuneVal val{best_pick[i].tx, best_vx, best_pick[i].tz, best_pf};
    batch_tune_cache().put(key, val);
  }
  B->dirty = true;
  ++B->version;
  if (best_ms) *best_ms = best_all;
  return SL_OK;
}

sl_status sl_batch_count(const sl_batch* B, int32_t* count) {
  if (!B || !count) return fail(SL_E_INVALID, "batch handle or count is NULL");
  *count = int32_t(B->runs.size());
  return SL_OK;
}

sl_status sl_batch_set_grid(sl_batch* B, int32_t workgroups) {
  if (!B) return fail(SL_E_INVALID, "batch handle is NULL");
  if (workgroups < 0 || workgroups > (1 << 24))
    return fail(SL_E_INVALID, "workgroups must be in [0, 2^24] (0: one per tile)");
  if (workgroups == B->grid_req) return SL_OK;
  B->grid_req = workgroups;
  B->dirty = true;
  ++B->version;
  return SL_OK;
}

sl_status sl_batch_get_grid(const sl_batch* B, int32_t* requested, int32_t* launched) {
  if (!B) return fail(SL_E_INVALID, "batch handle is NULL");
  long total = 0;
  for (const sl_lattice* L : B->runs) total += L->v.tile.nblocks();
  if (requested) *requested = B->grid_req;
  if (launched) *launched = B->runs.empty() ? 0 : batch_grid(B->grid_req, int(total));
  return SL_OK;
}

sl_status sl_batch_step(sl_batch* B, int64_t steps, double dt, int32_t order) {
  if (!B) return fail(SL_E_INVALID, "batch handle is NULL");
  if (steps < 0) return fail(SL_E_INVALID, "steps must be >= 0");
  if (!std::isfinite(dt)) return fail(SL_E_INVALID, "dt must be finite");
  const std::vector<double> w = weights_for(order);
  if (w.empty()) return fail(SL_E_INVALID, "order must be 2, 4, 6 or 8 (got %d)", order);
  if (B->runs.empty() || steps == 0) return SL_OK;
  for (sl_lattice* L : B->runs) {
    sl_status st = check_stable(L, dt, order);
    if (st != SL_OK) return st;
  }
  if (B->dirty) {
    sl_status st = batch_upload(B);
    if (st != SL_OK) return st;
  }
  // order after each member's own stream
  for (sl_lattice* L : B->runs) {
    if (L->stream == B->stream) continue;
    HIP_TRY(hipEventRecord(B->ev, L->stream));
    HIP_TRY(hipStreamWaitEvent(B->stream, B->ev, 0));
  }
  HIP_TRY(launch_batched_begin(B->run_dev, int(B->runs.size()), w[0], dt, B->stream));
  // Interior chunks of kBatchChunk steps replay one captured graph (kept
  // while dt, order and membership are unchanged, whatever the step count
  // of the call); the last 1 .. kBatchChunk steps launch eagerly.
  const int64_t chunks = (steps - 1) / kBatchChunk;
  if (chunks > 0) {
    if (!(B->gexec && B->g_dt == dt && B->g_order == order && B->g_version == B->version)) {
      batch_drop_graph(B);
      HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
      sl_status st = batch_enqueue(B, kBatchChunk, dt, w, false);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(B->stream, &g);
      if (st != SL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(SL_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
      B->graph = g;
      HIP_TRY(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
      B->g_dt = dt;
      B->g_order = order;
      B->g_version = B->version;
    }
    for (int64_t c = 0; c < chunks; ++c) HIP_TRY(hipGraphLaunch(B->gexec, B->stream));
  }
  {
    const sl_status st = batch_enqueue(B, steps - chunks * kBatchChunk, dt, w, true);
    if (st != SL_OK) return st;
  }
  // members' later work waits for the batch
  HIP_TRY(hipEventRecord(B->ev, B->stream));
  for (sl_lattice* L : B->runs) {
    if (L->stream == B->stream) continue;
    HIP_TRY(hipStreamWaitEvent(L->stream, B->ev, 0));
  }
  return SL_OK;
}

sl_status sl_batch_synchronize(sl_batch* B) {
  if (!B) return fail(SL_E_INVALID, "batch handle is NULL");
  HIP_TRY(hipStreamSynchronize(B->stream));
  for (sl_lattice* L : B->runs)
    if (L->stream != B->stream) HIP_TRY(hipStreamSynchronize(L->stream));
  if (B->runs.empty()) return SL_OK;
  if (B->dirty) {
    const sl_status st = batch_upload(B);
    if (st != SL_OK) return st;
  }
  // every member's scalars in one gather and one read-back
  const int R = int(B->runs.size());
  B->sc_host.resize(size_t(R));
  HIP_TRY(launch_gather_scalars(B->run_dev, R, B->sc_dev, B->stream));
  HIP_TRY(hipMemcpyAsync(B->sc_host.data(), B->sc_dev, sizeof(DevScalars) * R, hipMemcpyDeviceToHost,
                         B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  sl_status first = SL_OK;
  for (int r = 0; r < R; ++r) {
    const sl_status st = apply_scalars(B->runs[r], B->sc_host[r]);
    if (st != SL_OK && first == SL_OK) first = st;
  }
  return first;
}

sl_status sl_device_memory(size_t* free_bytes, size_t* total_bytes) {
  size_t f = 0, t = 0;
  HIP_TRY(hipMemGetInfo(&f, &t));
  if (free_bytes) *free_bytes = f;
  if (total_bytes) *total_bytes = t;
  return SL_OK;
}

}  // extern "C"
