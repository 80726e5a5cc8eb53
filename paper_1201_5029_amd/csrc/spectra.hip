// Energy- and number-density spectra of one field (the post-processing
// spectra of Sec. 2.4).  With F_n = DFT(phi_i)/n^3 and P_n = DFT(pi_i)/n^3 of
// the synchronised state, k_eff^2 of the lattice's stencil and m_eff^2 the
// lattice mean of d^2V/dphi_i^2:
//
//   rho_n   = |P_n|^2/(2 a^6) + (k_eff^2/(2 a^2 dx^2) + m_eff^2/2) |F_n|^2
//   omega_n = sqrt(k_eff^2/(a^2 dx^2) + m_eff^2),   n_n = rho_n / omega_n
//
// rho_n is mode n's share of the quadratic energy density (its sum over
// n != 0 is the fluctuations' kinetic, gradient and m_eff^2 energy), n_n the
// corresponding occupation density; both are binned like the field
// spectrum (|n| rounded half away from zero, n = 0 excluded).

#include "device.h"

namespace symlat {

namespace {

template <int KIND, int NF, typename T>
__device__ __forceinline__ void d2v_diag(const T (&f)[NF], const PotT<T>& P, T (&d)[NF]) {
  if constexpr (KIND == SL_POT_FREE) {
#pragma unroll
    for (int i = 0; i < NF; ++i) d[i] = P.p[i];
  } else if constexpr (KIND == SL_POT_CHAOTIC2) {
    d[0] = P.p[0] + P.p[1] * f[1] * f[1];
    d[1] = P.p[1] * f[0] * f[0];
  } else if constexpr (KIND == SL_POT_OSCILLON) {
    const T x2 = f[0] * f[0];
    d[0] = P.p[0] - T(3) * P.p[1] * x2 + T(5) * P.p[2] * x2 * x2;
  } else {
    const T m2 = P.p[0], K = P.p[1], invM2 = P.p[2];
    const T u = T(0.5) * (f[0] * f[0] + f[1] * f[1]);
    if (u > T(0)) {
      const T base = m2 * (T(1) + K + K * dev_log<T>(u * invM2));
      d[0] = base + m2 * K * f[0] * f[0] / u;
      d[1] = base + m2 * K * f[1] * f[1] / u;
    } else {
      d[0] = T(0);
      d[1] = T(0);
    }
  }
}

constexpr int kSpecBlocksMax = 256;

struct Bufs4 {
  const void* phi[2];
  const void* pi[2];
};

// Per-block compensated sums of d^2V/dphi_i^2 at the synchronised fields.
template <typename T, int NF, int KIND>
__global__ __launch_bounds__(kBlock) void meff_kernel(Bufs4 B, const DevScalars* sc, PotArgs prm,
                                                     size_t n3, size_t n2, int zs,
                                                     double* part) {
  __shared__ KSum scratch[4 * NF];
  const int par = sc->parity;
  const T* phi = static_cast<const T*>(B.phi[par]);
  const T* pi = static_cast<const T*>(B.pi[par]);
  const double c = sc->c_pend;
  PotT<double> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = prm.p[i];
  KSum acc[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) acc[i] = KSum{0.0, 0.0};
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    double f[NF], d[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const size_t o = field_site(i, e, zs, n2);
      f[i] = (sc->off_phi[i] + c * sc->off_pi[i]) + fma(c, double(pi[o]), double(phi[o]));
    }
    d2v_diag<KIND, NF, double>(f, pot, d);
#pragma unroll
    for (int i = 0; i < NF; ++i) kadd(acc[i], d[i]);
  }
  block_reduce<NF>(acc, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      part[(size_t(blockIdx.x) * NF + i) * 2] = acc[i].s;
      part[(size_t(blockIdx.x) * NF + i) * 2 + 1] = acc[i].c;
    }
  }
}

__global__ void meff_finalize_kernel(const double* part, int nblocks, int nf, double inv_n3,
                                     double* m2) {
  const int i = threadIdx.x;
  if (i >= nf) return;
  KSum t{0.0, 0.0};
  for (int b = 0; b < nblocks; ++b)
    t = kcombine(t, KSum{part[(size_t(b) * nf + i) * 2], part[(size_t(b) * nf + i) * 2 + 1]});
  m2[i] = (t.s + t.c) * inv_n3;
}

template <typename T>
__global__ void momentum_to_complex_kernel(Bufs4 B, const DevScalars* sc, size_t n3, size_t n2,
                                           int zs, int field, double2* F) {
  const T* pi = static_cast<const T*>(B.pi[sc->parity]);
  const double off = sc->off_pi[field];
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride)
    F[e] = make_double2(off + double(pi[field_site(field, e, zs, n2)]), 0.0);
}

__device__ __forceinline__ int shell_index(long long m) {
  long long b = (long long)floor(sqrt(double(m)));
  if (b * b > m) --b;
  if ((b + 1) * (b + 1) <= m) ++b;
  return int(m > b * b + b ? b + 1 : b);
}

// Per-block bin sums [5][nbins]: |F|^2, rho, n, |n|, count.
__global__ __launch_bounds__(kBlock) void mode_spectra_kernel(int n, const double2* __restrict__ F,
                                                             const double2* __restrict__ P,
                                                             int nbins, double inv_n6, Stencil st,
                                                             const DevScalars* sc, const double* m2p,
                                                             int field, double inv_dx2,
                                                             double* part) {
  extern __shared__ double sh[];
  for (int b = threadIdx.x; b < 5 * nbins; b += blockDim.x) sh[b] = 0.0;
  __syncthreads();
  const double a = sc->a;
  const double a2 = a * a, a6 = a2 * a2 * a2;
  const double m2 = m2p[field];
  const size_t n2 = size_t(n) * n, n3 = n2 * n;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    const int ux = int(e % n), uy = int((e / n) % n), uz = int(e / n2);
    const int kx = 2 * ux >= n ? ux - n : ux, ky = 2 * uy >= n ? uy - n : uy,
              kz = 2 * uz >= n ? uz - n : uz;
    const long long m = (long long)kx * kx + (long long)ky * ky + (long long)kz * kz;
    if (m == 0) continue;
    const int b = shell_index(m);
    if (b >= nbins) continue;
    double k2;
    if (st.kind == 0) {
      const double sx = sinpi(double(ux) / n), sy = sinpi(double(uy) / n), sz = sinpi(double(uz) / n);
      k2 = 4.0 * sz * sz + 4.0 * sy * sy + 4.0 * sx * sx;
    } else {
      const double cx = cospi(2.0 * ux / n), cy = cospi(2.0 * uy / n), cz = cospi(2.0 * uz / n);
      k2 = -(st.c[0] + 2.0 * st.c[1] * (cz + cy + cx) + 4.0 * st.c[2] * (cz * cy + cz * cx + cy * cx) +
             8.0 * st.c[3] * cz * cy * cx);
    }
    const double2 f = F[e], p = P[e];
    const double f2 = (f.x * f.x + f.y * f.y) * inv_n6;
    const double p2 = (p.x * p.x + p.y * p.y) * inv_n6;
    const double rho = p2 / (2.0 * a6) + (k2 * inv_dx2 / (2.0 * a2) + 0.5 * m2) * f2;
    const double w2 = k2 * inv_dx2 / a2 + m2;
    const double num = w2 > 0.0 ? rho / sqrt(w2) : 0.0;
    atomicAdd(&sh[b], f2);
    atomicAdd(&sh[nbins + b], rho);
    atomicAdd(&sh[2 * nbins + b], num);
    atomicAdd(&sh[3 * nbins + b], sqrt(double(m)));
    atomicAdd(&sh[4 * nbins + b], 1.0);
  }
  __syncthreads();
  double* out = part + size_t(blockIdx.x) * 5 * nbins;
  for (int b = threadIdx.x; b < 5 * nbins; b += blockDim.x) out[b] = sh[b];
}

// out5 = [k_b | <|F|^2>_b | <rho>_b | <n>_b | count_b], fixed block order.
__global__ void mode_spectra_finalize(const double* part, int nblocks, int nbins, double L,
                                      double* out5) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  KSum s[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  double cnt = 0.0;
  for (int q = 0; q < nblocks; ++q) {
    const double* r = part + size_t(q) * 5 * nbins;
    for (int k = 0; k < 4; ++k) kadd(s[k], r[k * nbins + b]);
    cnt += r[4 * nbins + b];
  }
  const double inv = cnt > 0 ? 1.0 / cnt : 0.0;
  out5[b] = 2.0 * M_PI * (s[3].s + s[3].c) * inv / L;
  out5[nbins + b] = (s[0].s + s[0].c) * inv;
  out5[2 * nbins + b] = (s[1].s + s[1].c) * inv;
  out5[3 * nbins + b] = (s[2].s + s[2].c) * inv;
  out5[4 * nbins + b] = cnt;
}

int spec_grid(size_t n3) {
  const size_t b = (n3 + kBlock - 1) / kBlock;
  return int(b < size_t(kSpecBlocksMax) ? b : kSpecBlocksMax);
}

Bufs4 bufs4(const LatView& v) {
  Bufs4 B;
  for (int k = 0; k < 2; ++k) {
    B.phi[k] = v.phi[k];
    B.pi[k] = v.pi[k];
  }
  return B;
}

template <typename T, int NF, int KIND>
hipError_t meff_t(const LatView& v, double* part, double* m2, hipStream_t s) {
  const size_t n3 = size_t(v.n) * v.n * v.n;
  const int nb = spec_grid(n3);
  hipLaunchKernelGGL((meff_kernel<T, NF, KIND>), dim3(nb), dim3(kBlock), 0, s, bufs4(v), v.sc, v.prm,
                     n3, size_t(v.n) * v.n, v.zs, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(meff_finalize_kernel, dim3(1), dim3(64), 0, s, part, nb, NF, 1.0 / double(n3), m2);
  return hipGetLastError();
}

template <typename T>
hipError_t meff_prec(const LatView& v, double* part, double* m2, hipStream_t s) {
  switch (v.pot) {
    case SL_POT_CHAOTIC2: return meff_t<T, 2, SL_POT_CHAOTIC2>(v, part, m2, s);
    case SL_POT_OSCILLON: return meff_t<T, 1, SL_POT_OSCILLON>(v, part, m2, s);
    case SL_POT_QBALL_LOG: return meff_t<T, 2, SL_POT_QBALL_LOG>(v, part, m2, s);
    default: break;
  }
  switch (v.nf) {
    case 1: return meff_t<T, 1, SL_POT_FREE>(v, part, m2, s);
    case 2: return meff_t<T, 2, SL_POT_FREE>(v, part, m2, s);
    case 3: return meff_t<T, 3, SL_POT_FREE>(v, part, m2, s);
    case 4: return meff_t<T, 4, SL_POT_FREE>(v, part, m2, s);
    case 5: return meff_t<T, 5, SL_POT_FREE>(v, part, m2, s);
    case 6: return meff_t<T, 6, SL_POT_FREE>(v, part, m2, s);
    case 7: return meff_t<T, 7, SL_POT_FREE>(v, part, m2, s);
    default: return meff_t<T, 8, SL_POT_FREE>(v, part, m2, s);
  }
}

}  // namespace

size_t meff_partial_doubles(int nf) { return size_t(kSpecBlocksMax) * 2 * nf; }

hipError_t launch_meff(const LatView& v, double* part, double* m2_dev, hipStream_t s) {
  return v.prec == SL_FP32 ? meff_prec<float>(v, part, m2_dev, s) : meff_prec<double>(v, part, m2_dev, s);
}

hipError_t launch_momentum_to_complex(const LatView& v, int field, double2* cbuf, hipStream_t s) {
  const size_t n3 = size_t(v.n) * v.n * v.n;
  const int nb = int((n3 + kBlock - 1) / kBlock < 65536 ? (n3 + kBlock - 1) / kBlock : 65536);
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(momentum_to_complex_kernel<float>, dim3(nb), dim3(kBlock), 0, s, bufs4(v), v.sc,
                       n3, size_t(v.n) * v.n, v.zs, field, cbuf);
  else
    hipLaunchKernelGGL(momentum_to_complex_kernel<double>, dim3(nb), dim3(kBlock), 0, s, bufs4(v), v.sc,
                       n3, size_t(v.n) * v.n, v.zs, field, cbuf);
  return hipGetLastError();
}

int mode_spectra_blocks(int n) { return spec_grid(size_t(n) * n * n); }

hipError_t launch_mode_spectra(const LatView& v, int field, const double2* F, const double2* P,
                               int nbins, double* part, const double* m2_dev, double* out5,
                               hipStream_t s) {
  const int nb = mode_spectra_blocks(v.n);
  const double n3 = double(v.n) * v.n * v.n;
  hipLaunchKernelGGL(mode_spectra_kernel, dim3(nb), dim3(kBlock), size_t(5) * nbins * sizeof(double), s,
                     v.n, F, P, nbins, 1.0 / (n3 * n3), v.st, v.sc, m2_dev, field, v.bg.inv_dx2, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mode_spectra_finalize, dim3((nbins + 255) / 256), dim3(256), 0, s, part, nb, nbins,
                     v.bg.L, out5);
  return hipGetLastError();
}

}  // namespace symlat
