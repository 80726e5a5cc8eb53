// The linearized integrator (Sec. 2.2 and Sec. 2.4): a homogeneous
// background (a, p_a, phi0_i, pi0_i) and field perturbations evolved in
// Fourier space, eq. (2.38), with the five-part splitting of eq. (2.49)
// composed as in eq. (2.50):
//
//   H1(t/2) H2(t/2) H3(t/2) H4(t/2) H5(t) H4(t/2) H3(t/2) H2(t/2) H1(t/2)
//
// H1-H3 move only the background; H4 drifts the perturbations
// (dPhi += dPi t/a^2), H5 kicks them (dPi -= (a^2 k_eff^2/dx^2 + a^4 H) dPhi t
// with H the Hessian of V at phi0); the perturbations do not act back on
// the background.  Every mode with the same k_eff^2 obeys the same linear
// equations, so, as the paper does, the map of each distinct class of modes
// is integrated once as growth functions -- the 2N x 2N matrix M(eta, k_eff)
// of eq. (2.51) -- and then applied to every mode of the lattice.
//
// Device design:
//  * modes are grouped by the multiset of folded wave numbers
//    {min(n_d, N - n_d)}: for every stencil of the cubic family k_eff^2 is a
//    symmetric function of them.  The classes are ranked combinatorially,
//    q = C(a+2,3) + C(b+1,2) + c for a >= b >= c, so a mode finds its class
//    without a table;
//  * the background is a short sequential ODE: one lane integrates it for a
//    chunk of stages and writes, per stage, the coefficients the growth
//    functions need (drift t/(2a^2), a^2 t/dx^2 and a^4 t H);
//  * the growth kernel gives one lane to each (class, column) of M: the
//    lane keeps one 2N-vector in registers and runs the whole chunk of
//    stages, reading the per-stage coefficients with wave-uniform loads.
//    This is FP64 ALU work with no memory traffic inside the loop;
//  * the apply kernel multiplies each Fourier mode by its class's M.
// All arithmetic is FP64.

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "device.h"
#include "timing.h"

namespace symlat {

namespace {

constexpr int kLinMaxFields = 4;
constexpr int kLinChunk = 512;   // stages per background-table chunk (two buffers)
// Growth-function columns per lane: the variants are 1, 2 and (one or two
// fields) a whole class of 2 NF columns.  More columns per lane share each
// coefficient load and give more independent chains; fewer give more waves.
// The handle times the variants on its first evolve call and keeps the
// fastest.
constexpr int kGrowthVariants = 3;
template <int NF>
constexpr int cols_variant(int v) { return v == 0 ? 1 : (v == 1 ? 2 : (NF <= 2 ? 2 * NF : 2)); }
constexpr int kMaxStages = 15;

struct LinScalars {
  double a, p_a, eta;
  double phi0[kLinMaxFields];
  double pi0[kLinMaxFields];
};

struct LinConsts {
  double inv6VLm2;  // 1/(6 V_L m_pl^2)
  double VL;        // V_L = n^3
  double VL_rho_r;  // V_L rho_gamma0
  double VL_rho_m;  // V_L rho_m0
  double inv_dx2;   // 1/dx^2
  double mpl2VL12;  // 12 V_L m_pl^2
  int32_t expand;
  int32_t pad;
};

struct Weights {
  double w[kMaxStages];
  int32_t s;
  int32_t pad;
};

__host__ __device__ inline long long c3(long long m) { return m * (m - 1) * (m - 2) / 6; }
__host__ __device__ inline long long c2(long long m) { return m * (m - 1) / 2; }

// Rank of the multiset {a >= b >= c >= 0}.
__host__ __device__ inline long long rank3(int a, int b, int c) {
  return c3(a + 2) + c2(b + 1) + c;
}

// Number of classes for side n: multisets of 3 values from 0..n/2.
inline long long class_count(int n) { return c3(n / 2 + 3); }

__device__ inline void unrank3(long long q, int hmax, int& a, int& b, int& c) {
  int lo = 0, hi = hmax;  // largest a with C(a+2,3) <= q
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (c3(mid + 2) <= q) lo = mid; else hi = mid - 1;
  }
  a = lo;
  q -= c3(a + 2);
  lo = 0;
  hi = a;  // largest b with C(b+1,2) <= q
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (c2(mid + 1) <= q) lo = mid; else hi = mid - 1;
  }
  b = lo;
  c = int(q - c2(b + 1));
}

__device__ inline int fold(int v, int n) { return v <= n - v ? v : n - v; }

__device__ inline long long class_of_mode(int nz, int ny, int nx, int n) {
  int a = fold(nz, n), b = fold(ny, n), c = fold(nx, n);
  if (a < b) { const int t = a; a = b; b = t; }
  if (b < c) { const int t = b; b = c; c = t; }
  if (a < b) { const int t = a; a = b; b = t; }
  return rank3(a, b, c);
}

// k_eff^2 of every class: minus the stencil's eigenvalue at k_d = 2 pi m_d/N.
__global__ void class_keff2_kernel(double* k2, long long ncls, int n, Stencil st) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncls) return;
  int a, b, c;
  unrank3(q, n / 2, a, b, c);
  double v;
  if (st.kind == 0) {
    const double sa = sinpi(double(a) / n), sb = sinpi(double(b) / n), sc = sinpi(double(c) / n);
    v = 4.0 * sa * sa + 4.0 * sb * sb + 4.0 * sc * sc;
  } else {
    const double ca = cospi(2.0 * a / n), cb = cospi(2.0 * b / n), cc = cospi(2.0 * c / n);
    v = -(st.c[0] + 2.0 * st.c[1] * (ca + cb + cc) + 4.0 * st.c[2] * (ca * cb + ca * cc + cb * cc) +
          8.0 * st.c[3] * ca * cb * cc);
  }
  k2[q] = v;
}

// Hessian d^2V/dphi_i dphi_j at a homogeneous point (row-major NF x NF).
template <int KIND, int NF>
__device__ void hessian(const double (&f)[NF], const PotT<double>& P, double (&H)[NF][NF]) {
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) H[i][j] = 0.0;
  if constexpr (KIND == SL_POT_FREE) {
#pragma unroll
    for (int i = 0; i < NF; ++i) H[i][i] = P.p[i];
  } else if constexpr (KIND == SL_POT_CHAOTIC2) {
    const double m2 = P.p[0], G = P.p[1];
    H[0][0] = m2 + G * f[1] * f[1];
    H[0][1] = H[1][0] = 2.0 * G * f[0] * f[1];
    H[1][1] = G * f[0] * f[0];
  } else if constexpr (KIND == SL_POT_OSCILLON) {
    const double m2 = P.p[0], lam = P.p[1], g = P.p[2];
    const double x2 = f[0] * f[0];
    H[0][0] = m2 - 3.0 * lam * x2 + 5.0 * g * x2 * x2;
  } else {
    const double m2 = P.p[0], K = P.p[1], invM2 = P.p[2];
    const double u = 0.5 * (f[0] * f[0] + f[1] * f[1]);
    if (u > 0.0) {
      const double base = m2 * (1.0 + K + K * log(u * invM2));
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) H[i][j] = (i == j ? base : 0.0) + m2 * K * f[i] * f[j] / u;
    }
  }
}

// p_a from the background constraint H^(0) = 0 (expanding branch).
template <int KIND, int NF>
__global__ void lin_constraint_kernel(LinScalars* S, LinConsts K, PotArgs prm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  PotT<double> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = prm.p[i];
  LinScalars s = *S;
  double f[NF], dV[NF], V, p2 = 0.0;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    f[i] = s.phi0[i];
    p2 += s.pi0[i] * s.pi0[i];
  }
  potential<KIND, NF, double>(f, pot, V, dV);
  const double a = s.a;
  const double E0 = K.VL * (p2 / (2.0 * a * a) + a * a * a * a * V) + K.VL_rho_r + a * K.VL_rho_m;
  s.p_a = K.expand ? -sqrt(K.mpl2VL12 * (E0 > 0.0 ? E0 : 0.0)) : 0.0;
  *S = s;
}

// One lane integrates the background through `steps` composed steps and
// writes the per-stage growth coefficients: tab[st * E + 0] = t/(2 a^2)
// (the H4 drift), [1] = -a^2 t/dx^2 (H5, times k_eff^2), [2 + i NF + j] =
// -a^4 t H_ij(phi0), with a and phi0 at the H4/H5 part of the stage (kick
// terms negated so the growth kernel applies them as fused multiply-adds).
template <int KIND, int NF>
__global__ void lin_table_kernel(LinScalars* S, LinConsts K, PotArgs prm, Weights W, double h,
                                 int steps, double* tab) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  constexpr int E = 2 + NF * NF;
  PotT<double> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = prm.p[i];
  LinScalars s = *S;
  double a = s.a, pa = s.p_a;
  double f[NF], q[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    f[i] = s.phi0[i];
    q[i] = s.pi0[i];
  }
  int k = 0;
  for (int step = 0; step < steps; ++step) {
    for (int j = 0; j < W.s; ++j, ++k) {
      const double tau = W.w[j] * h;
      const double half = 0.5 * tau;
      // H1(t/2)
      if (K.expand) a = a - pa * half * K.inv6VLm2;
      // H2(t/2)
      double p2 = 0.0;
#pragma unroll
      for (int i = 0; i < NF; ++i) p2 += q[i] * q[i];
      if (K.expand) pa = pa + K.VL * (p2 / (a * a * a)) * half - K.VL_rho_m * half;
      const double cdr = half / (a * a);
#pragma unroll
      for (int i = 0; i < NF; ++i) f[i] = f[i] + q[i] * cdr;
      // H3(t/2), twice around H4 H5 H4 (a and phi0 do not move in between)
      double V, dV[NF];
      potential<KIND, NF, double>(f, pot, V, dV);
      const double a2 = a * a, a4 = a2 * a2;
      double H[NF][NF];
      hessian<KIND, NF>(f, pot, H);
      double* t = tab + size_t(k) * E;
      t[0] = cdr;
      t[1] = -(a2 * tau * K.inv_dx2);
#pragma unroll
      for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int jj = 0; jj < NF; ++jj) t[2 + i * NF + jj] = -(a4 * tau * H[i][jj]);
      for (int rep = 0; rep < 2; ++rep) {
        if (K.expand) pa = pa - 4.0 * a2 * a * K.VL * V * half;
#pragma unroll
        for (int i = 0; i < NF; ++i) q[i] = q[i] - a4 * dV[i] * half;
      }
      // H2(t/2)
      p2 = 0.0;
#pragma unroll
      for (int i = 0; i < NF; ++i) p2 += q[i] * q[i];
      if (K.expand) pa = pa + K.VL * (p2 / (a * a * a)) * half - K.VL_rho_m * half;
#pragma unroll
      for (int i = 0; i < NF; ++i) f[i] = f[i] + q[i] * cdr;
      // H1(t/2)
      if (K.expand) a = a - pa * half * K.inv6VLm2;
    }
    s.eta = s.eta + h;
  }
  s.a = a;
  s.p_a = pa;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    s.phi0[i] = f[i];
    s.pi0[i] = q[i];
  }
  *S = s;
}

// Growth functions: lane (class q, columns c0 .. c0 + CPL - 1) holds those
// columns of M(q) -- each the evolved state that starts as its unit vector
// -- as NF field rows x and NF momentum rows p, and applies `nst` stages of
// drift-kick-drift.  The stage coefficients are wave-uniform; the next
// stage's are loaded while the current one computes, and CPL columns per
// lane share each load.
template <int NF, int CPL>
__global__ __launch_bounds__(kBlock) void lin_growth_kernel(double* __restrict__ M,
                                                            const double* __restrict__ k2,
                                                            long long ncls,
                                                            const double* __restrict__ tab,
                                                            int nst, int identity) {
  constexpr int R = 2 * NF;
  constexpr int E = 2 + NF * NF;
  constexpr int LPC = R / CPL;  // lanes per class
  static_assert(R % CPL == 0, "columns per lane must divide 2 NF");
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncls * LPC) return;
  const long long q = g / LPC;
  const int c0 = int(g - q * LPC) * CPL;
  double x[CPL][NF], p[CPL][NF];
  double* m = M + (q * R + c0) * R;
#pragma unroll
  for (int k = 0; k < CPL; ++k)
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      if (identity) {
        x[k][i] = (c0 + k == i) ? 1.0 : 0.0;
        p[k][i] = (c0 + k == NF + i) ? 1.0 : 0.0;
      } else {
        x[k][i] = m[k * R + i];
        p[k][i] = m[k * R + NF + i];
      }
    }
  const double kk = k2[q];
  double t[E];
#pragma unroll
  for (int e = 0; e < E; ++e) t[e] = tab[e];
  for (int st = 0; st < nst; ++st) {
    // next stage's coefficients (past the end: the last stage again)
    const double* tn = tab + size_t(st + 1 < nst ? st + 1 : st) * E;
    double u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = tn[e];
    const double c = t[0];
    const double ngk = t[1] * kk;  // -a^2 t k_eff^2 / dx^2
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
#pragma unroll
      for (int i = 0; i < NF; ++i) x[k][i] = fma(c, p[k][i], x[k][i]);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        double q = fma(ngk, x[k][i], p[k][i]);
#pragma unroll
        for (int j = 0; j < NF; ++j) q = fma(t[2 + i * NF + j], x[k][j], q);
        p[k][i] = q;
      }
#pragma unroll
      for (int i = 0; i < NF; ++i) x[k][i] = fma(c, p[k][i], x[k][i]);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) t[e] = u[e];
  }
#pragma unroll
  for (int k = 0; k < CPL; ++k)
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      m[k * R + i] = x[k][i];
      m[k * R + NF + i] = p[k][i];
    }
}

// Every Fourier mode times its class's M: (dPhi, dPi) <- M (dPhi, dPi).
template <int NF>
__global__ __launch_bounds__(kBlock) void lin_apply_kernel(double2* __restrict__ dphi,
                                                           double2* __restrict__ dpi,
                                                           const double* __restrict__ M, int n) {
  constexpr int R = 2 * NF;
  const size_t n2 = size_t(n) * n, n3 = n2 * n;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    const int x = int(e % n), y = int((e / n) % n), z = int(e / n2);
    const double* m = M + class_of_mode(z, y, x, n) * R * R;
    double2 u[R];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      u[i] = dphi[i * n3 + e];
      u[NF + i] = dpi[i * n3 + e];
    }
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = make_double2(0.0, 0.0);
#pragma unroll
    for (int col = 0; col < R; ++col)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double w = m[col * R + r];
        v[r].x = fma(w, u[col].x, v[r].x);
        v[r].y = fma(w, u[col].y, v[r].y);
      }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      dphi[i * n3 + e] = v[i];
      dpi[i * n3 + e] = v[NF + i];
    }
  }
}

__global__ void real_to_complex_kernel(const double* __restrict__ r, double2* __restrict__ c,
                                       size_t n3, double shift) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride)
    c[e] = make_double2(r[e] - shift, 0.0);
}

__global__ void complex_to_real_kernel(const double2* __restrict__ c, double* __restrict__ r,
                                       size_t n3, double scale, double add) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride)
    r[e] = fma(c[e].x, scale, add);
}

int grid_of(size_t work) {
  const size_t b = (work + kBlock - 1) / kBlock;
  return int(b < 65536 ? b : 65536);
}

// ---- dispatch over (potential family, fields) ------------------------------
struct LinFns {
  void (*constraint)(LinScalars*, LinConsts, PotArgs);
  void (*table)(LinScalars*, LinConsts, PotArgs, Weights, double, int, double*);
  void (*growth[kGrowthVariants])(double*, const double*, long long, const double*, int, int);
  int cols[kGrowthVariants];
  void (*apply)(double2*, double2*, const double*, int);
};

template <int KIND, int NF>
LinFns fns_t() {
  return LinFns{lin_constraint_kernel<KIND, NF>,
                lin_table_kernel<KIND, NF>,
                {lin_growth_kernel<NF, cols_variant<NF>(0)>, lin_growth_kernel<NF, cols_variant<NF>(1)>,
                 lin_growth_kernel<NF, cols_variant<NF>(2)>},
                {cols_variant<NF>(0), cols_variant<NF>(1), cols_variant<NF>(2)},
                lin_apply_kernel<NF>};
}

bool pick_lin(int kind, int nf, LinFns* out) {
  switch (kind) {
    case SL_POT_CHAOTIC2: *out = fns_t<SL_POT_CHAOTIC2, 2>(); return true;
    case SL_POT_OSCILLON: *out = fns_t<SL_POT_OSCILLON, 1>(); return true;
    case SL_POT_QBALL_LOG: *out = fns_t<SL_POT_QBALL_LOG, 2>(); return true;
    case SL_POT_FREE:
      switch (nf) {
        case 1: *out = fns_t<SL_POT_FREE, 1>(); return true;
        case 2: *out = fns_t<SL_POT_FREE, 2>(); return true;
        case 3: *out = fns_t<SL_POT_FREE, 3>(); return true;
        case 4: *out = fns_t<SL_POT_FREE, 4>(); return true;
        default: return false;
      }
    default: return false;
  }
}

}  // namespace
}  // namespace symlat

using namespace symlat;

struct sl_linear {
  sl_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t n3 = 0;
  long long ncls = 0;
  int pot_kind = -1;
  bool pot_set = false;
  bool state_set = false;
  double pot_raw[kMaxFields] = {0};
  PotArgs prm{};
  Stencil st{{-6.0, 1.0, 0.0, 0.0}, 0, 0};
  double keff2_max = 12.0;
  bool k2_valid = false;
  LinConsts K{};
  LinScalars host{};          // last background read back
  LinScalars* sc = nullptr;   // device background
  double2* dphi = nullptr;    // nf * n^3 modes of the field perturbations
  double2* dpi = nullptr;     // nf * n^3 modes of the momentum perturbations
  double* M = nullptr;        // ncls * (2 nf)^2 growth functions
  double* k2 = nullptr;       // ncls values of k_eff^2
  double* tab = nullptr;      // two buffers of kLinChunk stages of coefficients
  hipStream_t aux = nullptr;  // background-table stream, overlapped with growth
  hipEvent_t ev_tab[2] = {nullptr, nullptr};   // table chunk ready (per buffer)
  hipEvent_t ev_grow[2] = {nullptr, nullptr};  // growth chunk done with a buffer
  hipEvent_t ev_sync = nullptr;
  double* stage = nullptr;    // n^3 doubles of host<->device staging
  double2* fa = nullptr;      // transform scratch
  double2* fb = nullptr;
  double2* tw = nullptr;
  int growth_variant = -1;  // columns-per-lane variant, -1 until timed
  bool timing = false;
  // kind 0: one chunk (e0 -> e1 table on the aux stream, e2 -> e3 growth);
  // kind 1: the apply launch (e0 -> e1)
  struct Rec {
    hipEvent_t e[4];
    int kind;
  };
  std::vector<Rec> recs;
};

namespace {

void lin_free(sl_linear* L) {
  void* ptrs[] = {L->sc, L->dphi, L->dpi, L->M, L->k2, L->tab, L->stage, L->fa, L->fb, L->tw};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& r : L->recs)
    for (hipEvent_t e : r.e)
      if (e) (void)hipEventDestroy(e);
  L->recs.clear();
  for (int k = 0; k < 2; ++k) {
    if (L->ev_tab[k]) (void)hipEventDestroy(L->ev_tab[k]);
    if (L->ev_grow[k]) (void)hipEventDestroy(L->ev_grow[k]);
  }
  if (L->ev_sync) (void)hipEventDestroy(L->ev_sync);
  if (L->aux) (void)hipStreamDestroy(L->aux);
  if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
}

// Append a timing record; *index is its position in L->recs (indices stay
// valid as the vector grows).
sl_status new_rec(sl_linear* L, int kind, size_t* index) {
  sl_linear::Rec r{{nullptr, nullptr, nullptr, nullptr}, kind};
  const int ne = kind == 0 ? 4 : 2;
  for (int i = 0; i < ne; ++i) {
    if (timing_event_create(&r.e[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(r.e[j]);
      return fail(SL_E_DEVICE, "cannot create a timing event");
    }
  }
  L->recs.push_back(r);
  *index = L->recs.size() - 1;
  return SL_OK;
}

sl_status lin_read(sl_linear* L) {
  HIP_TRY(hipMemcpyAsync(&L->host, L->sc, sizeof(LinScalars), hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(hipStreamSynchronize(L->stream));
  if (!std::isfinite(L->host.a) || !std::isfinite(L->host.p_a))
    return fail(SL_E_NONFINITE, "the background became non-finite");
  return SL_OK;
}

// 3-D DFT fa -> fb (fa clobbered); sign -1 forward, +1 inverse (unnormalised).
sl_status lin_dft3(sl_linear* L, int sign) {
  const int n = L->cfg.n;
  HIP_TRY(launch_twiddles(n, sign, L->tw, L->stream));
  HIP_TRY(launch_dft_axis(n, L->fa, L->fb, L->tw, 0, L->stream));
  HIP_TRY(launch_dft_axis(n, L->fb, L->fa, L->tw, 1, L->stream));
  HIP_TRY(launch_dft_axis(n, L->fa, L->fb, L->tw, 2, L->stream));
  return SL_OK;
}

sl_status lin_keff2(sl_linear* L) {
  if (L->k2_valid) return SL_OK;
  hipLaunchKernelGGL(class_keff2_kernel, dim3(unsigned((L->ncls + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, L->stream, L->k2, L->ncls, L->cfg.n, L->st);
  HIP_TRY(hipGetLastError());
  L->k2_valid = true;
  return SL_OK;
}

double compensated_mean(const double* v, size_t n) {
  double s = 0.0, c = 0.0;
  for (size_t i = 0; i < n; ++i) {
    const double y = v[i] - c;
    const double t = s + y;
    c = (t - s) - y;
    s = t;
  }
  return s / double(n);
}

}  // namespace

extern "C" {

sl_status sl_linear_create(const sl_config* cfg, void* hip_stream, sl_linear** out) {
  if (!out) return fail(SL_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!config_ok(cfg, &why)) return fail(SL_E_INVALID, "invalid config: %s", why.c_str());
  if (cfg->nfields > kLinMaxFields)
    return fail(SL_E_INVALID, "the linearized integrator takes at most %d fields", kLinMaxFields);
  if (cfg->precision != SL_FP64)
    return fail(SL_E_INVALID, "the linearized integrator computes in FP64 only");
  sl_linear* L = new (std::nothrow) sl_linear();
  if (!L) return fail(SL_E_NOMEM, "host allocation failed");
  L->cfg = *cfg;
  const int n = cfg->n, nf = cfg->nfields;
  L->n3 = size_t(n) * n * n;
  L->ncls = class_count(n);
  if (hip_stream) {
    L->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess) {
      delete L;
      return fail(SL_E_DEVICE, "cannot create a HIP stream");
    }
    L->own_stream = true;
  }
  const double dx = cfg->L / n;
  const double VL = double(L->n3);
  L->K.inv6VLm2 = 1.0 / (6.0 * VL * cfg->mpl * cfg->mpl);
  L->K.VL = VL;
  L->K.VL_rho_r = VL * cfg->rho_rad0;
  L->K.VL_rho_m = VL * cfg->rho_mat0;
  L->K.inv_dx2 = 1.0 / (dx * dx);
  L->K.mpl2VL12 = 12.0 * VL * cfg->mpl * cfg->mpl;
  L->K.expand = cfg->expansion == SL_EXPAND_SELF ? 1 : 0;
  const size_t R = 2 * size_t(nf);
  bool ok = hipMalloc(reinterpret_cast<void**>(&L->sc), sizeof(LinScalars)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->dphi), nf * L->n3 * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->dpi), nf * L->n3 * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->M), size_t(L->ncls) * R * R * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->k2), size_t(L->ncls) * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->tab),
                       2 * size_t(kLinChunk) * (2 + nf * nf) * sizeof(double)) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&L->aux, hipStreamNonBlocking) == hipSuccess;
  for (int k = 0; k < 2 && ok; ++k) {
    ok = ok && hipEventCreateWithFlags(&L->ev_tab[k], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&L->ev_grow[k], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipEventCreateWithFlags(&L->ev_sync, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->stage), L->n3 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->fa), L->n3 * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->fb), L->n3 * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&L->tw), size_t(n) * sizeof(double2)) == hipSuccess;
  if (!ok) {
    lin_free(L);
    delete L;
    return fail(SL_E_NOMEM, "device allocation for the linearized integrator failed");
  }
  LinScalars s{};
  s.a = cfg->a0;
  L->host = s;
  (void)hipMemcpyAsync(L->sc, &s, sizeof s, hipMemcpyHostToDevice, L->stream);
  (void)hipMemsetAsync(L->dphi, 0, nf * L->n3 * sizeof(double2), L->stream);
  (void)hipMemsetAsync(L->dpi, 0, nf * L->n3 * sizeof(double2), L->stream);
  if (hipStreamSynchronize(L->stream) != hipSuccess) {
    lin_free(L);
    delete L;
    return fail(SL_E_DEVICE, "device initialisation failed");
  }
  *out = L;
  return SL_OK;
}

sl_status sl_linear_destroy(sl_linear* L) {
  if (!L) return SL_OK;
  (void)hipStreamSynchronize(L->stream);
  lin_free(L);
  delete L;
  return SL_OK;
}

sl_status sl_linear_set_potential(sl_linear* L, int32_t kind, const double* params,
                                  int32_t nparams) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  const int nf = L->cfg.nfields;
  const int want = nparams_for(kind, nf);
  if (want < 0) return fail(SL_E_INVALID, "unknown potential kind %d", kind);
  const int nfk = nfields_for(kind);
  if (nfk && nfk != nf)
    return fail(SL_E_INVALID, "potential %d needs %d fields, handle has %d", kind, nfk, nf);
  if (nparams != want) return fail(SL_E_INVALID, "potential %d needs %d parameters, got %d", kind, want, nparams);
  if (!params) return fail(SL_E_INVALID, "params is NULL");
  for (int i = 0; i < nparams; ++i)
    if (!std::isfinite(params[i])) return fail(SL_E_INVALID, "parameter %d is not finite", i);
  if (kind == SL_POT_QBALL_LOG && !(params[2] > 0.0)) return fail(SL_E_INVALID, "M^2 must be > 0");
  PotArgs dev{};
  for (int i = 0; i < nparams; ++i) {
    L->pot_raw[i] = params[i];
    dev.p[i] = params[i];
  }
  if (kind == SL_POT_QBALL_LOG) dev.p[2] = 1.0 / params[2];
  L->prm = dev;
  L->pot_kind = kind;
  L->pot_set = true;
  return SL_OK;
}

sl_status sl_linear_set_stencil(sl_linear* L, const double* c) {
  if (!L || !c) return fail(SL_E_INVALID, "handle or coefficients are NULL");
  double scale = 1.0;
  for (int k = 0; k < 4; ++k) {
    if (!std::isfinite(c[k])) return fail(SL_E_INVALID, "coefficient %d is not finite", k);
    scale += std::fabs(c[k]) * (k == 0 ? 1 : (k == 1 ? 6 : (k == 2 ? 12 : 8)));
  }
  if (std::fabs(c[0] + 6.0 * c[1] + 12.0 * c[2] + 8.0 * c[3]) > 1e-12 * scale ||
      std::fabs(c[1] + 4.0 * c[2] + 4.0 * c[3] - 1.0) > 1e-12 * scale)
    return fail(SL_E_INVALID, "stencil outside the cubic family of eq. (2.7)");
  const int kind = (c[0] == -6.0 && c[1] == 1.0 && c[2] == 0.0 && c[3] == 0.0) ? 0 : 1;
  L->st = Stencil{{c[0], c[1], c[2], c[3]}, kind, 0};
  double kmax = 0.0;
  for (int v = 0; v < 8; ++v) {
    const double cz = (v & 4) ? -1.0 : 1.0, cy = (v & 2) ? -1.0 : 1.0, cx = (v & 1) ? -1.0 : 1.0;
    const double sym = c[0] + 2.0 * c[1] * (cz + cy + cx) + 4.0 * c[2] * (cz * cy + cz * cx + cy * cx) +
                       8.0 * c[3] * cz * cy * cx;
    if (-sym > kmax) kmax = -sym;
  }
  L->keff2_max = kmax;
  L->k2_valid = false;
  return SL_OK;
}

sl_status sl_linear_set_fields(sl_linear* L, const double* phi, const double* pi, double p_a) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  if (!L->pot_set) return fail(SL_E_STATE, "no potential set");
  if (!phi || !pi) return fail(SL_E_INVALID, "phi/pi is NULL");
  const int nf = L->cfg.nfields;
  LinScalars s{};
  s.a = L->cfg.a0;
  s.eta = 0.0;
  s.p_a = p_a;
  for (int i = 0; i < nf; ++i) {
    s.phi0[i] = compensated_mean(phi + i * L->n3, L->n3);
    s.pi0[i] = compensated_mean(pi + i * L->n3, L->n3);
    if (!std::isfinite(s.phi0[i]) || !std::isfinite(s.pi0[i]))
      return fail(SL_E_INVALID, "fields must be finite");
  }
  const unsigned gr = unsigned(grid_of(L->n3));
  for (int arr = 0; arr < 2; ++arr) {
    const double* src = arr == 0 ? phi : pi;
    double2* dst = arr == 0 ? L->dphi : L->dpi;
    for (int i = 0; i < nf; ++i) {
      HIP_TRY(hipMemcpyAsync(L->stage, src + i * L->n3, L->n3 * sizeof(double), hipMemcpyHostToDevice,
                             L->stream));
      hipLaunchKernelGGL(real_to_complex_kernel, dim3(gr), dim3(kBlock), 0, L->stream, L->stage, L->fa,
                         L->n3, arr == 0 ? s.phi0[i] : s.pi0[i]);
      HIP_TRY(hipGetLastError());
      sl_status st = lin_dft3(L, -1);
      if (st != SL_OK) return st;
      HIP_TRY(hipMemcpyAsync(dst + i * L->n3, L->fb, L->n3 * sizeof(double2), hipMemcpyDeviceToDevice,
                             L->stream));
      // the perturbation has zero lattice sum: its k = 0 mode is zero
      HIP_TRY(hipMemsetAsync(dst + i * L->n3, 0, sizeof(double2), L->stream));
    }
  }
  HIP_TRY(hipMemcpyAsync(L->sc, &s, sizeof s, hipMemcpyHostToDevice, L->stream));
  if (std::isnan(p_a)) {
    LinFns f;
    if (!pick_lin(L->pot_kind, nf, &f)) return fail(SL_E_INVALID, "unsupported potential/field count");
    hipLaunchKernelGGL(f.constraint, dim3(1), dim3(64), 0, L->stream, L->sc, L->K, L->prm);
    HIP_TRY(hipGetLastError());
  }
  sl_status st = lin_read(L);
  if (st != SL_OK) return st;
  L->state_set = true;
  return SL_OK;
}

sl_status sl_linear_evolve(sl_linear* L, int64_t steps, double dt, int32_t order) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  if (!L->state_set) return fail(SL_E_STATE, "no state (call sl_linear_set_fields)");
  if (steps < 0) return fail(SL_E_INVALID, "steps must be >= 0");
  if (!std::isfinite(dt)) return fail(SL_E_INVALID, "dt must be finite");
  const std::vector<double> w = weights_for(order);
  if (w.empty()) return fail(SL_E_INVALID, "order must be 2, 4, 6 or 8 (got %d)", order);
  const int nf = L->cfg.nfields;
  {
    double d2[kMaxFields];
    double m2max = 0.0;
    if (hessian_diag(L->pot_kind, nf, L->pot_raw, L->host.phi0, d2))
      for (int i = 0; i < nf; ++i) m2max = d2[i] > m2max ? d2[i] : m2max;
    const double dx = L->cfg.L / L->cfg.n;
    const double omax = std::sqrt(L->keff2_max / (dx * dx) + L->host.a * L->host.a * m2max);
    const double lim = stability_limit_for(order);
    if (omax * std::fabs(dt) > lim)
      return fail(SL_E_UNSTABLE, "omega_max*|dt| = %.4f exceeds the order-%d stability limit %.4f",
                  omax * std::fabs(dt), order, lim);
  }
  if (steps == 0) return SL_OK;
  LinFns f;
  if (!pick_lin(L->pot_kind, nf, &f)) return fail(SL_E_INVALID, "unsupported potential/field count");
  sl_status st = lin_keff2(L);
  if (st != SL_OK) return st;
  Weights W{};
  W.s = int(w.size());
  for (int j = 0; j < W.s; ++j) W.w[j] = w[j];
  const int E = 2 + nf * nf;
  const int steps_per_chunk = kLinChunk / W.s;
  auto grid_for_variant = [&](int v) {
    const long long lanes = L->ncls * (2 * nf / f.cols[v]);
    return unsigned((lanes + kBlock - 1) / kBlock);
  };
  const int nchunks = int((steps + steps_per_chunk - 1) / steps_per_chunk);
  // The background runs ahead on the aux stream, one chunk of stages into
  // one of two coefficient buffers; growth chunk k waits for table k, and
  // table k + 2 waits for growth k (it reuses that buffer).
  HIP_TRY(hipEventRecord(L->ev_sync, L->stream));
  HIP_TRY(hipStreamWaitEvent(L->aux, L->ev_sync, 0));
  std::vector<size_t> recs(nchunks, 0);
  auto enqueue_table = [&](int c) -> sl_status {
    const int64_t s0 = int64_t(c) * steps_per_chunk;
    const int k = int(steps - s0 < steps_per_chunk ? steps - s0 : steps_per_chunk);
    if (c >= 2) HIP_TRY(hipStreamWaitEvent(L->aux, L->ev_grow[c & 1], 0));
    if (L->timing) {
      sl_status s2 = new_rec(L, 0, &recs[c]);
      if (s2 != SL_OK) return s2;
      HIP_TRY(hipEventRecord(L->recs[recs[c]].e[0], L->aux));
    }
    hipLaunchKernelGGL(f.table, dim3(1), dim3(64), 0, L->aux, L->sc, L->K, L->prm, W, dt, k,
                       L->tab + size_t(c & 1) * kLinChunk * E);
    HIP_TRY(hipGetLastError());
    if (L->timing) HIP_TRY(hipEventRecord(L->recs[recs[c]].e[1], L->aux));
    HIP_TRY(hipEventRecord(L->ev_tab[c & 1], L->aux));
    return SL_OK;
  };
  st = enqueue_table(0);
  if (st != SL_OK) return st;
  for (int c = 0; c < nchunks; ++c) {
    if (c + 1 < nchunks) {
      st = enqueue_table(c + 1);
      if (st != SL_OK) return st;
    }
    const int64_t s0 = int64_t(c) * steps_per_chunk;
    const int k = int(steps - s0 < steps_per_chunk ? steps - s0 : steps_per_chunk);
    HIP_TRY(hipStreamWaitEvent(L->stream, L->ev_tab[c & 1], 0));
    const double* tb = L->tab + size_t(c & 1) * kLinChunk * E;
    if (c == 0 && L->growth_variant < 0) {
      // first call: time each variant on chunk 0, which starts from the
      // identity, so repeating it leaves the same M (every variant applies
      // the same operations to a column)
      hipEvent_t t0, t1;
      HIP_TRY(timing_event_create(&t0));
      HIP_TRY(timing_event_create(&t1));
      float best = 1e30f;
      int win = 1;
      hipError_t err = hipSuccess;
      // best of three launches per variant, variants interleaved, so that a
      // slow first launch does not decide
      for (int rep = 0; rep < 3 && err == hipSuccess; ++rep)
        for (int v = 0; v < kGrowthVariants && err == hipSuccess; ++v) {
          err = hipEventRecord(t0, L->stream);
          if (err == hipSuccess) {
            hipLaunchKernelGGL(f.growth[v], dim3(grid_for_variant(v)), dim3(kBlock), 0, L->stream,
                               L->M, L->k2, L->ncls, tb, k * W.s, 1);
            err = hipGetLastError();
          }
          if (err == hipSuccess) err = hipEventRecord(t1, L->stream);
          if (err == hipSuccess) err = hipEventSynchronize(t1);
          float ms = 0.0f;
          if (err == hipSuccess) err = hipEventElapsedTime(&ms, t0, t1);
          if (err == hipSuccess && ms < best) {
            best = ms;
            win = v;
          }
        }
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      if (err != hipSuccess) return fail(SL_E_DEVICE, "growth variant timing: %s", hipGetErrorString(err));
      L->growth_variant = win;
    }
    const int gv = L->growth_variant;
    if (L->timing) HIP_TRY(hipEventRecord(L->recs[recs[c]].e[2], L->stream));
    hipLaunchKernelGGL(f.growth[gv], dim3(grid_for_variant(gv)), dim3(kBlock), 0, L->stream, L->M,
                       L->k2, L->ncls, tb, k * W.s, c == 0 ? 1 : 0);
    HIP_TRY(hipGetLastError());
    if (L->timing) HIP_TRY(hipEventRecord(L->recs[recs[c]].e[3], L->stream));
    HIP_TRY(hipEventRecord(L->ev_grow[c & 1], L->stream));
  }
  // later work on the handle's stream sees the final background
  HIP_TRY(hipEventRecord(L->ev_sync, L->aux));
  HIP_TRY(hipStreamWaitEvent(L->stream, L->ev_sync, 0));
  hipEvent_t a0 = nullptr, a1 = nullptr;
  if (L->timing) {
    size_t r = 0;
    st = new_rec(L, 1, &r);
    if (st != SL_OK) return st;
    a0 = L->recs[r].e[0];
    a1 = L->recs[r].e[1];
    HIP_TRY(hipEventRecord(a0, L->stream));
  }
  hipLaunchKernelGGL(f.apply, dim3(unsigned(grid_of(L->n3))), dim3(kBlock), 0, L->stream, L->dphi,
                     L->dpi, L->M, L->cfg.n);
  HIP_TRY(hipGetLastError());
  if (L->timing) HIP_TRY(hipEventRecord(a1, L->stream));
  return SL_OK;
}

sl_status sl_linear_get_fields(sl_linear* L, double* phi_out, double* pi_out) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  if (!L->state_set) return fail(SL_E_STATE, "no state");
  sl_status st = lin_read(L);
  if (st != SL_OK) return st;
  const int nf = L->cfg.nfields;
  const unsigned gr = unsigned(grid_of(L->n3));
  const double inv = 1.0 / double(L->n3);
  for (int arr = 0; arr < 2; ++arr) {
    double* out = arr == 0 ? phi_out : pi_out;
    if (!out) continue;
    const double2* src = arr == 0 ? L->dphi : L->dpi;
    for (int i = 0; i < nf; ++i) {
      HIP_TRY(hipMemcpyAsync(L->fa, src + i * L->n3, L->n3 * sizeof(double2), hipMemcpyDeviceToDevice,
                             L->stream));
      st = lin_dft3(L, +1);
      if (st != SL_OK) return st;
      hipLaunchKernelGGL(complex_to_real_kernel, dim3(gr), dim3(kBlock), 0, L->stream, L->fb, L->stage,
                         L->n3, inv, arr == 0 ? L->host.phi0[i] : L->host.pi0[i]);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(out + i * L->n3, L->stage, L->n3 * sizeof(double), hipMemcpyDeviceToHost,
                             L->stream));
    }
  }
  HIP_TRY(hipStreamSynchronize(L->stream));
  return SL_OK;
}

sl_status sl_linear_get_background(sl_linear* L, double* eta, double* a, double* p_a, double* phi0,
                                   double* pi0) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  sl_status st = lin_read(L);
  if (st != SL_OK) return st;
  if (eta) *eta = L->host.eta;
  if (a) *a = L->host.a;
  if (p_a) *p_a = L->host.p_a;
  for (int i = 0; i < L->cfg.nfields; ++i) {
    if (phi0) phi0[i] = L->host.phi0[i];
    if (pi0) pi0[i] = L->host.pi0[i];
  }
  return SL_OK;
}

sl_status sl_linear_classes(sl_linear* L, int64_t* nclasses) {
  if (!L || !nclasses) return fail(SL_E_INVALID, "handle or output is NULL");
  *nclasses = L->ncls;
  return SL_OK;
}

sl_status sl_linear_synchronize(sl_linear* L) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  return lin_read(L);
}

sl_status sl_linear_set_kernel_timing(sl_linear* L, int32_t enable) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(L->stream));
  for (auto& r : L->recs)
    for (hipEvent_t e : r.e)
      if (e) (void)hipEventDestroy(e);
  L->recs.clear();
  L->timing = enable != 0;
  return SL_OK;
}

sl_status sl_linear_kernel_timing(sl_linear* L, int64_t* growth_launches, double* growth_ms,
                                  double* table_ms, double* apply_ms) {
  if (!L) return fail(SL_E_INVALID, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(L->stream));
  double g = 0.0, t = 0.0, ap = 0.0;
  long long ng = 0;
  for (auto& r : L->recs) {
    float ms = 0.0f;
    if (r.kind == 0) {
      HIP_TRY(hipEventElapsedTime(&ms, r.e[0], r.e[1]));
      t += ms;
      HIP_TRY(hipEventElapsedTime(&ms, r.e[2], r.e[3]));
      g += ms;
      ++ng;
    } else {
      HIP_TRY(hipEventElapsedTime(&ms, r.e[0], r.e[1]));
      ap += ms;
    }
    for (hipEvent_t e : r.e)
      if (e) (void)hipEventDestroy(e);
  }
  L->recs.clear();
  if (growth_launches) *growth_launches = ng;
  if (growth_ms) *growth_ms = g;
  if (table_ms) *table_ms = t;
  if (apply_ms) *apply_ms = ap;
  return SL_OK;
}

}  // extern "C"
