// Device helpers shared by the lattice kernels: compensated FP64 sums,
// fixed-order wave/workgroup reductions, the potential families and the
// field drift.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace symlat {

// ---------------------------------------------------------------------------
// Compensated summation.  A running sum is a pair (s, c) whose exact value is
// s + c; values are added with Knuth's branch-free TwoSum so that the FP64
// result is insensitive to the magnitude order of the terms.  All trees
// below combine pairs in a fixed order, so sums are bitwise reproducible.
// ---------------------------------------------------------------------------
struct KSum {
  double s, c;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  double bp = s - a;
  double ap = s - bp;
  e = (a - ap) + (b - bp);
}

__device__ __forceinline__ void kadd(KSum& k, double x) {
#pragma clang fp contract(off)
  double s, e;
  two_sum(k.s, x, s, e);
  k.s = s;
  k.c += e;
}

__device__ __forceinline__ KSum kcombine(KSum a, KSum b) {
#pragma clang fp contract(off)
  KSum r;
  double e;
  two_sum(a.s, b.s, r.s, e);
  r.c = (a.c + b.c) + e;
  return r;
}

// Butterfly over the 64 lanes of a wavefront (fixed xor pattern).
__device__ __forceinline__ KSum wave_reduce(KSum v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    KSum o;
    o.s = __shfl_xor(v.s, off, 64);
    o.c = __shfl_xor(v.c, off, 64);
    v = kcombine(v, o);
  }
  return v;
}

// Offset of site e = (z n + y) n + x of field i in a field array whose
// planes are zs n^2 elements apart (the fields of a plane one after the
// other, x fastest).
__device__ __forceinline__ size_t field_site(int i, size_t e, int zs, size_t n2) {
  const size_t z = e / n2;
  return (z * size_t(zs) + size_t(i)) * n2 + (e - z * n2);
}

// Reduce NV pairs over a 256-thread workgroup; thread 0 gets the result.
// scratch: 4 * NV KSum of LDS.  Contains barriers: all threads must call.
template <int NV>
__device__ __forceinline__ void block_reduce(KSum (&v)[NV], KSum* scratch) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_reduce(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) scratch[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      KSum t = scratch[k];
      for (int w = 1; w < kBlock / 64; ++w) t = kcombine(t, scratch[w * NV + k]);
      v[k] = t;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Potential families (program units); V once per site, dV per field.
// ---------------------------------------------------------------------------
template <typename T>
struct PotT {
  T p[kMaxFields];
};

template <typename T>
__device__ __forceinline__ T dev_log(T x);
template <>
__device__ __forceinline__ float dev_log<float>(float x) { return logf(x); }
template <>
__device__ __forceinline__ double dev_log<double>(double x) { return log(x); }

template <int KIND, int NF, typename T>
__device__ __forceinline__ void potential(const T (&f)[NF], const PotT<T>& P, T& V, T (&dV)[NF]) {
  if constexpr (KIND == SL_POT_FREE) {
    V = T(0);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      dV[i] = P.p[i] * f[i];
      V += T(0.5) * dV[i] * f[i];
    }
  } else if constexpr (KIND == SL_POT_CHAOTIC2) {
    static_assert(NF == 2, "two fields");
    const T m2 = P.p[0], G = P.p[1];
    const T f2 = f[0] * f[0], c2 = f[1] * f[1];
    const T mc = m2 + G * c2;
    V = T(0.5) * f2 * mc;
    dV[0] = f[0] * mc;
    dV[1] = G * f2 * f[1];
  } else if constexpr (KIND == SL_POT_OSCILLON) {
    static_assert(NF == 1, "one field");
    const T m2 = P.p[0], lam = P.p[1], g = P.p[2];
    const T x = f[0], x2 = x * x;
    // V = x^2 (m2/2 - lam x^2/4 + g x^4/6),  dV = x (m2 - lam x^2 + g x^4)
    V = x2 * (T(0.5) * m2 + x2 * (T(-0.25) * lam + x2 * (g * T(1.0 / 6.0))));
    dV[0] = x * (m2 + x2 * (-lam + x2 * g));
  } else {
    static_assert(NF == 2, "two fields");
    const T m2 = P.p[0], K = P.p[1], invM2 = P.p[2];  // p[2] holds 1/M^2
    const T u = T(0.5) * (f[0] * f[0] + f[1] * f[1]);
    if (u > T(0)) {
      const T lg = dev_log<T>(u * invM2);
      V = m2 * u * (T(1) + K * lg);
      const T fac = m2 * (T(1) + K + K * lg);
      dV[0] = fac * f[0];
      dV[1] = fac * f[1];
    } else {
      V = T(0);
      dV[0] = T(0);
      dV[1] = T(0);
    }
  }
}

// Constants of the difference form below that depend only on the offsets
// (uniform over a pass): for the Q-ball family u0 = (fb_0^2 + fb_1^2)/2, its
// reciprocal, ln(u0/M^2) and dV(fb).
template <typename T>
struct SplitK {
  T u0, inv_u0, L0, dv0[2];
  bool has_u0;
};

template <int KIND, int NF, typename T>
__device__ __forceinline__ SplitK<T> split_consts(const double (&fb)[NF], const PotArgs& prm) {
  SplitK<T> k{};
  if constexpr (KIND == SL_POT_QBALL_LOG) {
    const double u0 = 0.5 * (fb[0] * fb[0] + fb[1] * fb[1]);
    k.has_u0 = u0 > 0.0;
    k.u0 = T(u0);
    k.inv_u0 = k.has_u0 ? T(1.0 / u0) : T(0);
    const double L0 = k.has_u0 ? log(u0 * prm.p[2]) : 0.0;
    k.L0 = T(L0);
    const double g0 = k.has_u0 ? prm.p[0] * (1.0 + prm.p[1] + prm.p[1] * L0) : 0.0;
    k.dv0[0] = T(g0 * fb[0]);
    k.dv0[1] = T(g0 * fb[1]);
  }
  return k;
}

// V at fb + d and dV(fb + d) - dV(fb), for FP32 remainders d around FP64
// offsets fb: each difference is written as d times a factor (algebraic
// identities of the family), so that it keeps the relative precision of d
// instead of cancelling two values near dV(fb).  V is formed from the full
// values (it only enters FP64 lattice sums).
template <int KIND, int NF, typename T>
__device__ __forceinline__ void potential_split(const T (&fb)[NF], const T (&d)[NF],
                                                const PotT<T>& P, const SplitK<T>& k, T& V,
                                                T (&ddV)[NF]) {
  T x[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) x[i] = fb[i] + d[i];
  if constexpr (KIND == SL_POT_FREE) {
    V = T(0);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      ddV[i] = P.p[i] * d[i];
      V += T(0.5) * (P.p[i] * x[i]) * x[i];
    }
  } else if constexpr (KIND == SL_POT_CHAOTIC2) {
    // dV0 = phi (m2 + G chi^2), dV1 = G phi^2 chi
    const T m2 = P.p[0], G = P.p[1];
    const T f2 = x[0] * x[0], c2 = x[1] * x[1];
    const T mc = m2 + G * c2;
    V = T(0.5) * f2 * mc;
    const T dc2 = d[1] * (T(2) * fb[1] + d[1]);  // chi^2 - chi0^2
    const T df2 = d[0] * (T(2) * fb[0] + d[0]);  // phi^2 - phi0^2
    ddV[0] = d[0] * mc + fb[0] * (G * dc2);
    ddV[1] = G * (f2 * d[1] + fb[1] * df2);
  } else if constexpr (KIND == SL_POT_OSCILLON) {
    // dV = m2 x - lam x^3 + g x^5; x^k - b^k = d sum_j x^j b^(k-1-j)
    const T m2 = P.p[0], lam = P.p[1], g = P.p[2];
    const T xx = x[0], b = fb[0], x2 = xx * xx, b2 = b * b, xb = xx * b;
    V = x2 * (T(0.5) * m2 + x2 * (T(-0.25) * lam + x2 * (g * T(1.0 / 6.0))));
    const T s3 = x2 + xb + b2;
    const T s5 = x2 * x2 + xb * (x2 + b2) + x2 * b2 + b2 * b2;
    ddV[0] = d[0] * (m2 - lam * s3 + g * s5);
  } else {
    // V = m2 u (1 + K ln(u/M^2)), dV_i = m2 phi_i g(u), g = 1 + K + K ln(u/M^2):
    // dV_i(x) - dV_i(fb) = m2 (d_i g(u) + fb_i K ln(u/u0))
    const T m2 = P.p[0], K = P.p[1], invM2 = P.p[2];
    const T u = T(0.5) * (x[0] * x[0] + x[1] * x[1]);
    if (!(u > T(0))) {
      V = T(0);
      ddV[0] = -k.dv0[0];
      ddV[1] = -k.dv0[1];
    } else if (k.has_u0) {
      // r = ln(u/u0) = ln(1 + q), q = (u - u0)/u0 formed from the remainders:
      // w = 1 + q rounded, e = q - (w - 1) exactly (Fast2Sum, |q| <= 1), and
      // ln(1 + q) = ln(w) + e/w + O(e^2), with 1/w ~ 2 - w (|e| <= 2^-24);
      // far below u0 the log of u/u0 itself, one log per site either way
      const T du = fb[0] * d[0] + fb[1] * d[1] + T(0.5) * (d[0] * d[0] + d[1] * d[1]);
      const T q = du * k.inv_u0;
      const bool near = q > T(-0.5) && q < T(1);
      const T w = T(1) + q;
      const T e = q - (w - T(1));
      const T r = logf(near ? w : u * k.inv_u0) + (near ? e * (T(2) - w) : T(0));
      const T Lu = k.L0 + r;
      V = m2 * u * (T(1) + K * Lu);
      const T gu = T(1) + K + K * Lu;
      ddV[0] = m2 * (d[0] * gu + fb[0] * (K * r));
      ddV[1] = m2 * (d[1] * gu + fb[1] * (K * r));
    } else {
      const T lg = logf(u * invM2);
      V = m2 * u * (T(1) + K * lg);
      const T gu = m2 * (T(1) + K + K * lg);
      ddV[0] = gu * x[0];
      ddV[1] = gu * x[1];
    }
  }
}

// Field drift phi + c pi as one fused multiply-add, so every tile computes
// the same value for a site.
__device__ __forceinline__ float drift(float phi, float pi, float c) { return fmaf(c, pi, phi); }
__device__ __forceinline__ double drift(double phi, double pi, double c) { return fma(c, pi, phi); }

__device__ __forceinline__ bool dev_finite(double x) { return !(isnan(x) || isinf(x)); }

}  // namespace symlat
