// The hot path: one fused stage pass of the composed symplectic map and the
// device-side scalar update that follows it.
//
// Stage j of a composition (weight w_j, Sec. 2.3 eq. (2.45)) is the
// second-order map eq. (2.48):  H1(w_j h/2) H2(w_j h/2) H3(w_j h) H2(w_j h/2)
// H1(w_j h/2), with the exact flows of eq. (2.47).  Between two kicks the
// momenta are constant, so the two H2 field drifts around a merged H1 are one
// update phi += c pi with c = w_j h/(2 a_j^2) + w_{j+1} h/(2 a_{j+1}^2).  The
// pass therefore applies "drift owed, then kick":
//
//   phi~ = phi + c pi                       (at every site and halo point)
//   pi'  = pi + alpha D[phi~] - beta dV(phi~),  alpha = a^2 w h/dx^2,
//                                               beta  = a^4 w h
//
// and sums, in FP64 with compensation, the lattice quantities the background
// flows need: sum phi~ D phi~ and sum V (for the H3 kick of p_a) and
// sum pi'^2 (for the H2 kicks of p_a).  The global sums make every stage a
// grid-wide dependency, so a stage is one pass plus one small finalize.
//
// Data layout: phi and pi are [field][z][y][x] (x fastest) in two ping-pong
// buffers; the pass reads buffer `parity` and writes the other one, so no
// tile ever reads a value another tile has already advanced.
//
// Tiling: a 256-thread workgroup owns a TX x TY column tile (TX lanes of a
// wavefront along x, coalesced) and marches up TZ planes in z.  Each thread
// keeps phi~ at z-1, z, z+1 of its own column in registers; the current
// plane goes to LDS (double-buffered) with a one-cell periodic halo in x and
// y so the four in-plane neighbours come from LDS.  Halo cells are loaded
// and drifted by designated threads.

#include "device.h"

namespace symlat {

namespace {

struct PassParams {
  const void* phi[2];
  const void* pi[2];
  void* phi_w[2];
  void* pi_w[2];
  const DevScalars* sc;
  double* partials;
  PotArgs prm;
  int n;
  int tx, logtx, ty, tz;
  int ntx, nty, ntz;
};

template <typename T, int NF, int KIND>
__global__ __launch_bounds__(kBlock) void pass_kernel(PassParams P) {
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  __shared__ KSum red_scratch[4 * 3];

  const int par = P.sc->parity;
  const T* __restrict__ phi_in = static_cast<const T*>(P.phi[par]);
  const T* __restrict__ pi_in = static_cast<const T*>(P.pi[par]);
  T* __restrict__ phi_out = static_cast<T*>(P.phi_w[par ^ 1]);
  T* __restrict__ pi_out = static_cast<T*>(P.pi_w[par ^ 1]);
  const T c = static_cast<T>(P.sc->c_next);
  const T alpha = static_cast<T>(P.sc->alpha);
  const T beta = static_cast<T>(P.sc->beta);
  PotT<T> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = static_cast<T>(P.prm.p[i]);

  const int n = P.n;
  const size_t n2 = size_t(n) * n;
  const size_t n3 = n2 * n;

  // tile of this workgroup (x tiles fastest, then y, then z chunks)
  int b = blockIdx.x;
  const int xt = b % P.ntx;
  b /= P.ntx;
  const int yt = b % P.nty;
  const int zt = b / P.nty;
  const int x0 = xt * P.tx, y0 = yt * P.ty, z0 = zt * P.tz;
  const int wx = min(P.tx, n - x0), wy = min(P.ty, n - y0), zc = min(P.tz, n - z0);

  const int tid = threadIdx.x;
  const int tx = tid & (P.tx - 1);
  const int ty = tid >> P.logtx;
  const bool active = (tx < wx) && (ty < wy);
  const int LX = P.tx + 2;
  const int plane = LX * (P.ty + 2);
  const int own = (ty + 1) * LX + (tx + 1);
  const size_t col = size_t(y0 + ty) * n + (x0 + tx);

  // halo job of this thread: -1 if none
  int hl = -1;
  size_t hcol = 0;
  {
    const int TX = P.tx, TY = P.ty;
    int hx = 0, hy = 0;
    if (tid < TX) {
      if (tid < wx) { hx = x0 + tid; hy = (y0 - 1 + n) % n; hl = tid + 1; }
    } else if (tid < 2 * TX) {
      const int t = tid - TX;
      if (t < wx) { hx = x0 + t; hy = (y0 + wy) % n; hl = (wy + 1) * LX + t + 1; }
    } else if (tid < 2 * TX + TY) {
      const int r = tid - 2 * TX;
      if (r < wy) { hx = (x0 - 1 + n) % n; hy = y0 + r; hl = (r + 1) * LX; }
    } else if (tid < 2 * TX + 2 * TY) {
      const int r = tid - 2 * TX - TY;
      if (r < wy) { hx = (x0 + wx) % n; hy = y0 + r; hl = (r + 1) * LX + wx + 1; }
    }
    hcol = size_t(hy) * n + hx;
  }

  KSum acc_dd{0.0, 0.0}, acc_v{0.0, 0.0}, acc_p{0.0, 0.0};
  T fm[NF], fc[NF], fp[NF], pc[NF], pp[NF];

  if (active) {
    const int zm = (z0 - 1 + n) % n;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const size_t om = i * n3 + size_t(zm) * n2 + col;
      const size_t oc = i * n3 + size_t(z0) * n2 + col;
      fm[i] = drift(phi_in[om], pi_in[om], c);
      pc[i] = pi_in[oc];
      fc[i] = drift(phi_in[oc], pc[i], c);
    }
  }

  int buf = 0;
  for (int z = z0; z < z0 + zc; ++z) {
    const int zp = (z + 1 == n) ? 0 : z + 1;
    if (active) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const size_t op = i * n3 + size_t(zp) * n2 + col;
        pp[i] = pi_in[op];
        fp[i] = drift(phi_in[op], pp[i], c);
      }
    }
    T* L = lds + size_t(buf) * NF * plane;
    if (hl >= 0) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const size_t oh = i * n3 + size_t(z) * n2 + hcol;
        L[i * plane + hl] = drift(phi_in[oh], pi_in[oh], c);
      }
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < NF; ++i) L[i * plane + own] = fc[i];
    }
    __syncthreads();
    if (active) {
      T D[NF], dV[NF], V;
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const T* Li = L + i * plane;
        D[i] = ((Li[own - 1] + Li[own + 1]) + (Li[own - LX] + Li[own + LX])) + (fm[i] + fp[i]) -
               T(6) * fc[i];
      }
      potential<KIND, NF, T>(fc, pot, V, dV);
      const size_t oc = size_t(z) * n2 + col;
      double dd = 0.0, p2 = 0.0;
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const T pn = pc[i] + alpha * D[i] - beta * dV[i];
        phi_out[i * n3 + oc] = fc[i];
        pi_out[i * n3 + oc] = pn;
        dd += double(fc[i]) * double(D[i]);
        p2 += double(pn) * double(pn);
      }
      kadd(acc_dd, dd);
      kadd(acc_v, double(V));
      kadd(acc_p, p2);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        fm[i] = fc[i];
        fc[i] = fp[i];
        pc[i] = pp[i];
      }
    }
    buf ^= 1;
  }

  KSum v[3] = {acc_dd, acc_v, acc_p};
  block_reduce<3>(v, red_scratch);
  if (threadIdx.x == 0) {
    double* out = P.partials + size_t(blockIdx.x) * 6;
    out[0] = v[0].s; out[1] = v[0].c;
    out[2] = v[1].s; out[3] = v[1].c;
    out[4] = v[2].s; out[5] = v[2].c;
  }
}

// ---------------------------------------------------------------------------
// Scalar updates.  They are written once and shared by the finalize and the
// begin kernel so that the operation sequence (hence every rounding) is the
// same whether a stage boundary falls inside one evolve call or between two.
// ---------------------------------------------------------------------------

// End of stage j: H3(w h) kick of p_a, H2(w h/2) kick of p_a, owed drift
// c = (w h/2)/a^2 of that H2, then H1(w h/2).
__device__ void end_stage(DevScalars& S, const BgConsts& K, double w, double h, double SdD,
                          double SV, double S2) {
#pragma clang fp contract(off)
  const double a = S.a_kick;
  const double tau = w * h;
  const double half = 0.5 * tau;
  if (K.expand) {
    const double S3 = a * SdD * K.inv_dx2 - 4.0 * a * a * a * SV;
    S.S3_last = S3;
    double pa = S.p_a + S3 * tau;
    pa = pa + (S2 / (a * a * a) - K.VL_rho_m) * half;
    S.p_a = pa;
    S.a = a - pa * half * K.inv6VLm2;
  } else {
    S.a = a;
  }
  S.S2 = S2;
  S.c_pend = half / (a * a);
}

// Begin of stage with weight w: H1(w h/2), H2(w h/2) kick of p_a, total drift
// owed before the kick, and the kick coefficients.
__device__ void begin_stage(DevScalars& S, const BgConsts& K, double w, double h) {
#pragma clang fp contract(off)
  const double tau = w * h;
  const double half = 0.5 * tau;
  double a = S.a;
  if (K.expand) {
    a = a - S.p_a * half * K.inv6VLm2;
    S.p_a = S.p_a + (S.S2 / (a * a * a) - K.VL_rho_m) * half;
  }
  S.a = a;
  S.c_next = S.c_pend + half / (a * a);
  S.c_pend = 0.0;
  S.a_kick = a;
  S.alpha = a * a * tau * K.inv_dx2;
  S.beta = a * a * a * a * tau;
}

__global__ __launch_bounds__(kBlock) void stage_finalize_kernel(DevScalars* sc, const double* partials,
                                                               int nblocks, BgConsts K, double w,
                                                               double w_next, double h, int has_next,
                                                               int end_of_step) {
  __shared__ KSum scratch[4 * 3];
  KSum v[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    const double* p = partials + size_t(b) * 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = kcombine(v[k], KSum{p[2 * k], p[2 * k + 1]});
  }
  block_reduce<3>(v, scratch);
  if (threadIdx.x == 0) {
    DevScalars S = *sc;
    const double SdD = v[0].s + v[0].c;
    const double SV = v[1].s + v[1].c;
    const double S2 = v[2].s + v[2].c;
    end_stage(S, K, w, h, SdD, SV, S2);
    S.parity ^= 1;
    if (end_of_step) S.eta = S.eta + h;
    if (has_next) begin_stage(S, K, w_next, h);
    if (!(dev_finite(SdD) && dev_finite(SV) && dev_finite(S2) && dev_finite(S.a) &&
          dev_finite(S.p_a)))
      S.status |= kStatusNonFinite;
    *sc = S;
  }
}

__global__ void begin_kernel(DevScalars* sc, BgConsts K, double w, double h) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    DevScalars S = *sc;
    begin_stage(S, K, w, h);
    *sc = S;
  }
}

template <typename T, int NF, int KIND>
hipError_t launch_pass_t(const LatView& v, hipStream_t s) {
  PassParams P;
  for (int k = 0; k < 2; ++k) {
    P.phi[k] = v.phi[k];
    P.pi[k] = v.pi[k];
    P.phi_w[k] = v.phi[k];
    P.pi_w[k] = v.pi[k];
  }
  P.sc = v.sc;
  P.partials = v.partials;
  P.prm = v.prm;
  P.n = v.n;
  P.tx = v.tile.tx;
  P.logtx = v.tile.logtx;
  P.ty = v.tile.ty;
  P.tz = v.tile.tz;
  P.ntx = v.tile.ntx;
  P.nty = v.tile.nty;
  P.ntz = v.tile.ntz;
  const size_t lds = size_t(2) * NF * (P.tx + 2) * (P.ty + 2) * sizeof(T);
  hipLaunchKernelGGL((pass_kernel<T, NF, KIND>), dim3(v.tile.nblocks()), dim3(kBlock), lds, s, P);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_pass(const LatView& v, hipStream_t s) {
  switch (v.pot) {
    case SL_POT_CHAOTIC2: return launch_pass_t<T, 2, SL_POT_CHAOTIC2>(v, s);
    case SL_POT_OSCILLON: return launch_pass_t<T, 1, SL_POT_OSCILLON>(v, s);
    case SL_POT_QBALL_LOG: return launch_pass_t<T, 2, SL_POT_QBALL_LOG>(v, s);
    default: break;
  }
  switch (v.nf) {
    case 1: return launch_pass_t<T, 1, SL_POT_FREE>(v, s);
    case 2: return launch_pass_t<T, 2, SL_POT_FREE>(v, s);
    case 3: return launch_pass_t<T, 3, SL_POT_FREE>(v, s);
    case 4: return launch_pass_t<T, 4, SL_POT_FREE>(v, s);
    case 5: return launch_pass_t<T, 5, SL_POT_FREE>(v, s);
    case 6: return launch_pass_t<T, 6, SL_POT_FREE>(v, s);
    case 7: return launch_pass_t<T, 7, SL_POT_FREE>(v, s);
    case 8: return launch_pass_t<T, 8, SL_POT_FREE>(v, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_pass(const LatView& v, hipStream_t s) {
  return v.prec == SL_FP32 ? dispatch_pass<float>(v, s) : dispatch_pass<double>(v, s);
}

hipError_t launch_stage_finalize(const LatView& v, double w, double w_next, double h, int has_next,
                                 int end_of_step, hipStream_t s) {
  hipLaunchKernelGGL(stage_finalize_kernel, dim3(1), dim3(kBlock), 0, s, v.sc, v.partials,
                     v.tile.nblocks(), v.bg, w, w_next, h, has_next, end_of_step);
  return hipGetLastError();
}

hipError_t launch_begin(const LatView& v, double w, double h, hipStream_t s) {
  hipLaunchKernelGGL(begin_kernel, dim3(1), dim3(64), 0, s, v.sc, v.bg, w, h);
  return hipGetLastError();
}

}  // namespace symlat
