// Initial state and field spectrum on the device.
//
// Random numbers: counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014:
// the k-th output from a seed is the published finaliser applied to
// seed + k * 0x9E3779B97F4A7C15) with 53-bit uniforms in (0, 1] and
// Box-Muller normals.  Draw r (0/1) of component c (0/1) for field i at
// linear index idx of an N-entry array uses output number
// 4 (i N + idx) + 2c + r + 1, so results do not depend on the launch shape.
//
// Transforms: separable 1-D DFTs along x, y, z, each output a length-n dot
// product with a twiddle table held in LDS (n <= 1024).  This is initial-state
// and diagnostic work, not the per-step path.

#include "device.h"

namespace symlat {

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform01(uint64_t seed, uint64_t counter) {
  const uint64_t x = splitmix64(seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull);
  return (double((x >> 11)) + 1.0) * 0x1.0p-53;
}

__device__ __forceinline__ double normal(uint64_t seed, uint64_t field, uint64_t count,
                                         uint64_t idx, uint64_t comp) {
  const uint64_t base = 4ull * (field * count + idx) + 2ull * comp;
  const double u1 = uniform01(seed, base);
  const double u2 = uniform01(seed, base + 1ull);
  return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

template <typename T>
__global__ void fill_homogeneous_kernel(void* phi0, void* pi0, int nf, int zs, size_t n2,
                                        size_t n3, PotArgs v0, PotArgs p0, Offsets off) {
  T* phi = static_cast<T*>(phi0);
  T* pi = static_cast<T*>(pi0);
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3 * nf; e += stride) {
    const int i = int(e / n3);  // field i, site e - i n^3
    const size_t d = field_site(i, e - size_t(i) * n3, zs, n2);
    phi[d] = static_cast<T>(v0.p[i] - off.phi[i]);
    pi[d] = static_cast<T>(p0.p[i] - off.pi[i]);
  }
}

// f_n for every mode n of one field: E|f_n|^2 = A^2/(2 omega_n L^3),
// omega_n^2 = k_eff^2/dx^2 + m_eff^2, f_0 = 0, f_{-n} = conj(f_n), real on
// self-conjugate modes; each +-n pair draws at its smaller linear index.
// k_eff^2 is minus the eigenvalue of the lattice Laplacian on the mode: for
// the 7-point stencil sum_d 4 sin^2(pi n_d/N), for a general member of the
// cubic family -(c0 + 2 c1 sum cos + 4 c2 sum cos cos + 8 c3 prod cos).
__global__ void vacuum_modes_kernel(double2* F, int n, double L, int field, double m2eff,
                                    double amp, uint64_t seed, Stencil st) {
  const size_t n2 = size_t(n) * n, n3 = n2 * n;
  const double dx = L / n;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    const int nx = int(e % n), ny = int((e / n) % n), nz = int(e / n2);
    const int mx = (n - nx) % n, my = (n - ny) % n, mz = (n - nz) % n;
    const size_t neg = (size_t(mz) * n + my) * n + mx;
    const size_t canon = e < neg ? e : neg;
    double keff2;
    if (st.kind == 0) {
      const double sx = sinpi(double(nx) / n), sy = sinpi(double(ny) / n), sz = sinpi(double(nz) / n);
      keff2 = 4.0 * sz * sz + 4.0 * sy * sy + 4.0 * sx * sx;
    } else {
      const double cx = cospi(2.0 * nx / n), cy = cospi(2.0 * ny / n), cz = cospi(2.0 * nz / n);
      keff2 = -(st.c[0] + 2.0 * st.c[1] * (cz + cy + cx) +
                4.0 * st.c[2] * (cz * cy + cz * cx + cy * cx) + 8.0 * st.c[3] * cz * cy * cx);
    }
    const double w2 = keff2 / (dx * dx) + m2eff;
    double P = 0.0;
    if (w2 > 0.0 && e != 0) P = amp * amp / (2.0 * sqrt(w2) * L * L * L);
    const double g1 = normal(seed, uint64_t(field), n3, canon, 0);
    double2 f;
    if (neg == e) {
      f.x = sqrt(P) * g1;
      f.y = 0.0;
    } else {
      const double g2 = normal(seed, uint64_t(field), n3, canon, 1);
      const double s = sqrt(P / 2.0);
      f.x = s * g1;
      f.y = (e == canon) ? s * g2 : -(s * g2);
    }
    F[e] = f;
  }
}

__global__ void twiddle_kernel(int n, int sign, double2* tw) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    const double t = 2.0 * double(m) / n;
    tw[m] = make_double2(cospi(t), sign * sinpi(t));
  }
}

// out[line, k] = sum_j in[line, j] tw[(j k) mod n] along `axis`.
__global__ __launch_bounds__(kBlock) void dft_axis_kernel(int n, const double2* __restrict__ in,
                                                         double2* __restrict__ out,
                                                         const double2* __restrict__ tw,
                                                         int axis) {
  extern __shared__ double2 stw[];
  for (int m = threadIdx.x; m < n; m += blockDim.x) stw[m] = tw[m];
  __syncthreads();
  const size_t n2 = size_t(n) * n, n3 = n2 * n;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const size_t stride = axis == 0 ? 1 : (axis == 1 ? size_t(n) : n2);
  const int k = int((e / stride) % n);
  const size_t base = e - size_t(k) * stride;
  double re = 0.0, im = 0.0;
  int m = 0;
  for (int j = 0; j < n; ++j) {
    const double2 a = in[base + size_t(j) * stride];
    const double2 w = stw[m];
    re += a.x * w.x - a.y * w.y;
    im += a.x * w.y + a.y * w.x;
    m += k;
    if (m >= n) m -= n;
  }
  out[e] = make_double2(re, im);
}

// The same transform for n = 2^L by the Stockham radix-2 recursion: for
// sub-transform size m = 1, 2, .., n/2 (l = n / 2m), the pairs x[k + j m]
// and x[k + j m + n/2] (j < l, k < m) give y[k + 2 j m] = sum and
// y[k + 2 j m + m] = tw[j m] (difference); after L stages the output is in
// natural order.  A workgroup loads `lines` whole lines into LDS (for the y
// and z axes, `lines` neighbouring columns x, so the loads are coalesced),
// runs the stages between two LDS buffers and writes the lines back.
__global__ __launch_bounds__(kBlock) void fft_axis_kernel(int n, int logn, int lines,
                                                         const double2* __restrict__ in,
                                                         double2* __restrict__ out,
                                                         const double2* __restrict__ tw,
                                                         int axis) {
  extern __shared__ double2 sbuf[];  // two buffers of lines * n values
  const int tid = int(threadIdx.x);
  const size_t n2 = size_t(n) * n;
  const int total = lines * n;
  size_t base, jstride, lstride;
  if (axis == 0) {  // rows: line-major and contiguous
    base = size_t(blockIdx.x) * total;
    jstride = 1;
    lstride = size_t(n);
  } else {          // `lines` neighbouring x at one z (axis 1) or one y (axis 2)
    const int groups = n / lines;
    const int xg = int(blockIdx.x % unsigned(groups)), other = int(blockIdx.x / unsigned(groups));
    lstride = 1;
    jstride = axis == 1 ? size_t(n) : n2;
    base = (axis == 1 ? size_t(other) * n2 : size_t(other) * n) + size_t(xg) * lines;
  }
  double2* x = sbuf;
  double2* y = sbuf + total;
  for (int idx = tid; idx < total; idx += kBlock) {
    int l, j;
    if (axis == 0) {
      l = idx >> logn;
      j = idx & (n - 1);
    } else {
      j = idx / lines;
      l = idx - j * lines;
    }
    x[l * n + j] = in[base + size_t(l) * lstride + size_t(j) * jstride];
  }
  __syncthreads();
  const int half = n >> 1;
  for (int s = 0; s < logn; ++s) {
    const int m = 1 << s;
    for (int b = tid; b < lines * half; b += kBlock) {
      const int line = b >> (logn - 1), t = b & (half - 1);
      const int j = t >> s, k = t & (m - 1);
      const double2 w = tw[j * m];
      const double2 c0 = x[line * n + k + j * m], c1 = x[line * n + k + j * m + half];
      const double dr = c0.x - c1.x, di = c0.y - c1.y;
      y[line * n + k + 2 * j * m] = make_double2(c0.x + c1.x, c0.y + c1.y);
      y[line * n + k + 2 * j * m + m] = make_double2(w.x * dr - w.y * di, w.x * di + w.y * dr);
    }
    __syncthreads();
    double2* t2 = x;
    x = y;
    y = t2;
  }
  for (int idx = tid; idx < total; idx += kBlock) {
    int l, j;
    if (axis == 0) {
      l = idx >> logn;
      j = idx & (n - 1);
    } else {
      j = idx / lines;
      l = idx - j * lines;
    }
    out[base + size_t(l) * lstride + size_t(j) * jstride] = x[l * n + j];
  }
}

template <typename T>
__global__ void add_real_kernel(void* phi0, const double2* F, size_t n3, size_t n2, int zs,
                                int field, double base, double scale) {
  T* phi = static_cast<T*>(phi0);
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride)
    phi[field_site(field, e, zs, n2)] = static_cast<T>(base + scale * F[e].x);
}

__global__ __launch_bounds__(kBlock) void white_kernel(double* g, size_t n3, int field,
                                                      uint64_t seed, double* partials) {
  __shared__ KSum scratch[4];
  KSum acc[1] = {{0.0, 0.0}};
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    const double v = normal(seed, uint64_t(field), n3, e, 0);
    g[e] = v;
    kadd(acc[0], v);
  }
  block_reduce<1>(acc, scratch);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = acc[0].s;
    partials[2 * blockIdx.x + 1] = acc[0].c;
  }
}

__global__ __launch_bounds__(kBlock) void mean_finalize_kernel(const double* partials, int nblocks,
                                                              double inv_count, double* mean) {
  __shared__ KSum scratch[4];
  KSum v[1] = {{0.0, 0.0}};
  for (int b = threadIdx.x; b < nblocks; b += kBlock)
    v[0] = kcombine(v[0], KSum{partials[2 * b], partials[2 * b + 1]});
  block_reduce<1>(v, scratch);
  if (threadIdx.x == 0) *mean = (v[0].s + v[0].c) * inv_count;
}

template <typename T>
__global__ void white_store_kernel(void* phi0, const double* g, const double* mean, size_t n3,
                                   size_t n2, int zs, int field, double base, double amp) {
  T* phi = static_cast<T*>(phi0);
  const double mu = *mean;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride)
    phi[field_site(field, e, zs, n2)] = static_cast<T>(base + amp * (g[e] - mu));
}

template <typename T>
__global__ void field_to_complex_kernel(const void* const phi_b0, const void* const phi_b1,
                                        const void* const pi_b0, const void* const pi_b1,
                                        const DevScalars* sc, size_t n3, size_t n2, int zs,
                                        int field, double2* F) {
  const int par = sc->parity;
  const T* phi = static_cast<const T*>(par ? phi_b1 : phi_b0);
  const T* pi = static_cast<const T*>(par ? pi_b1 : pi_b0);
  const double c = sc->c_pend;
  const double offp = sc->off_phi[field] + c * sc->off_pi[field];
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    const size_t d = field_site(field, e, zs, n2);
    F[e] = make_double2(offp + fma(c, double(pi[d]), double(phi[d])), 0.0);
  }
}

// Shell index of |n|^2 = m: round(|n|) half away from zero, in integers.
__device__ __forceinline__ int shell_of(long long m) {
  long long b = (long long)floor(sqrt(double(m)));
  if (b * b > m) --b;
  if ((b + 1) * (b + 1) <= m) ++b;
  return int(m > b * b + b ? b + 1 : b);
}

__global__ __launch_bounds__(kBlock) void spectrum_bins_kernel(int n, const double2* __restrict__ F,
                                                              int nbins, double inv_n6,
                                                              double* part) {
  extern __shared__ double sh[];  // [3][nbins]: sum |F|^2, sum |n|, count
  for (int b = threadIdx.x; b < 3 * nbins; b += blockDim.x) sh[b] = 0.0;
  __syncthreads();
  const size_t n2 = size_t(n) * n, n3 = n2 * n;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    int kx = int(e % n), ky = int((e / n) % n), kz = int(e / n2);
    if (2 * kx >= n) kx -= n;
    if (2 * ky >= n) ky -= n;
    if (2 * kz >= n) kz -= n;
    const long long m = (long long)kx * kx + (long long)ky * ky + (long long)kz * kz;
    if (m == 0) continue;
    const int b = shell_of(m);
    if (b >= nbins) continue;
    const double2 f = F[e];
    atomicAdd(&sh[b], (f.x * f.x + f.y * f.y) * inv_n6);
    atomicAdd(&sh[nbins + b], sqrt(double(m)));
    atomicAdd(&sh[2 * nbins + b], 1.0);
  }
  __syncthreads();
  double* out = part + size_t(blockIdx.x) * 3 * nbins;
  for (int b = threadIdx.x; b < 3 * nbins; b += blockDim.x) out[b] = sh[b];
}

__global__ void spectrum_finalize_kernel(const double* part, int nblocks, int nbins, double L,
                                         double* out3) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  KSum p{0.0, 0.0}, k{0.0, 0.0};
  double cnt = 0.0;
  for (int q = 0; q < nblocks; ++q) {
    const double* r = part + size_t(q) * 3 * nbins;
    kadd(p, r[b]);
    kadd(k, r[nbins + b]);
    cnt += r[2 * nbins + b];
  }
  const double P = p.s + p.c, K = k.s + k.c;
  out3[b] = cnt > 0 ? 2.0 * M_PI * (K / cnt) / L : 0.0;
  out3[nbins + b] = cnt > 0 ? P / cnt : 0.0;
  out3[2 * nbins + b] = cnt;
}

int grid_for(size_t count) {
  size_t nb = (count + kBlock - 1) / kBlock;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  return int(nb);
}

}  // namespace

hipError_t launch_fill_homogeneous(const LatView& v, const double* phi0, const double* pi0,
                                   const Offsets& off, hipStream_t s) {
  PotArgs a{}, b{};
  for (int i = 0; i < v.nf; ++i) {
    a.p[i] = phi0[i];
    b.p[i] = pi0[i];
  }
  const size_t n3 = size_t(v.n) * v.n * v.n;
  const int nb = grid_for(n3 * v.nf);
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(fill_homogeneous_kernel<float>, dim3(nb), dim3(kBlock), 0, s, v.phi[0],
                       v.pi[0], v.nf, v.zs, size_t(v.n) * v.n, n3, a, b, off);
  else
    hipLaunchKernelGGL(fill_homogeneous_kernel<double>, dim3(nb), dim3(kBlock), 0, s, v.phi[0],
                       v.pi[0], v.nf, v.zs, size_t(v.n) * v.n, n3, a, b, off);
  return hipGetLastError();
}

hipError_t launch_vacuum_modes(const LatView& v, double2* cbuf, int field, double m2eff,
                               double amp, uint64_t seed, hipStream_t s) {
  const size_t n3 = size_t(v.n) * v.n * v.n;
  hipLaunchKernelGGL(vacuum_modes_kernel, dim3(grid_for(n3)), dim3(kBlock), 0, s, cbuf, v.n,
                     v.bg.L, field, m2eff, amp, seed, v.st);
  return hipGetLastError();
}

hipError_t launch_twiddles(int n, int sign, double2* tw, hipStream_t s) {
  hipLaunchKernelGGL(twiddle_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, sign, tw);
  return hipGetLastError();
}

hipError_t launch_dft_axis(int n, const double2* in, double2* out, const double2* tw, int axis,
                           hipStream_t s) {
  if (n >= 2 && (n & (n - 1)) == 0) {
    // power of two: the radix-2 kernel, lines * n <= 2048 (two 32 KB LDS
    // buffers) and at most n lines, so that the y and z axes group whole
    // columns
    int logn = 0;
    while ((1 << logn) < n) ++logn;
    int lines = 2048 / n;
    if (lines > n) lines = n;
    if (lines < 1) lines = 1;
    const unsigned nb = unsigned(size_t(n) * n / lines);
    hipLaunchKernelGGL(fft_axis_kernel, dim3(nb), dim3(kBlock),
                       size_t(2) * lines * n * sizeof(double2), s, n, logn, lines, in, out, tw,
                       axis);
    return hipGetLastError();
  }
  const size_t n3 = size_t(n) * n * n;
  const size_t nb = (n3 + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(dft_axis_kernel, dim3(unsigned(nb)), dim3(kBlock), size_t(n) * sizeof(double2),
                     s, n, in, out, tw, axis);
  return hipGetLastError();
}

hipError_t launch_add_real(const LatView& v, const double2* cbuf, int field, double base,
                           double scale, hipStream_t s) {
  const size_t n3 = size_t(v.n) * v.n * v.n;
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(add_real_kernel<float>, dim3(grid_for(n3)), dim3(kBlock), 0, s, v.phi[0],
                       cbuf, n3, size_t(v.n) * v.n, v.zs, field, base, scale);
  else
    hipLaunchKernelGGL(add_real_kernel<double>, dim3(grid_for(n3)), dim3(kBlock), 0, s, v.phi[0],
                       cbuf, n3, size_t(v.n) * v.n, v.zs, field, base, scale);
  return hipGetLastError();
}

hipError_t launch_white(const LatView& v, double* gbuf, double* mean_dev, int field, double base,
                        double amp, uint64_t seed, hipStream_t s) {
  const size_t n3 = size_t(v.n) * v.n * v.n;
  const int nb = grid_for(n3) > 1024 ? 1024 : grid_for(n3);
  hipLaunchKernelGGL(white_kernel, dim3(nb), dim3(kBlock), 0, s, gbuf, n3, field, seed,
                     v.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mean_finalize_kernel, dim3(1), dim3(kBlock), 0, s, v.partials, nb,
                     1.0 / double(n3), mean_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(white_store_kernel<float>, dim3(grid_for(n3)), dim3(kBlock), 0, s,
                       v.phi[0], gbuf, mean_dev, n3, size_t(v.n) * v.n, v.zs, field, base, amp);
  else
    hipLaunchKernelGGL(white_store_kernel<double>, dim3(grid_for(n3)), dim3(kBlock), 0, s,
                       v.phi[0], gbuf, mean_dev, n3, size_t(v.n) * v.n, v.zs, field, base, amp);
  return hipGetLastError();
}

hipError_t launch_field_to_complex(const LatView& v, int field, double2* cbuf, hipStream_t s) {
  const size_t n3 = size_t(v.n) * v.n * v.n;
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(field_to_complex_kernel<float>, dim3(grid_for(n3)), dim3(kBlock), 0, s,
                       v.phi[0], v.phi[1], v.pi[0], v.pi[1], v.sc, n3, size_t(v.n) * v.n, v.zs,
                       field, cbuf);
  else
    hipLaunchKernelGGL(field_to_complex_kernel<double>, dim3(grid_for(n3)), dim3(kBlock), 0, s,
                       v.phi[0], v.phi[1], v.pi[0], v.pi[1], v.sc, n3, size_t(v.n) * v.n, v.zs,
                       field, cbuf);
  return hipGetLastError();
}

int spectrum_blocks(int n) {
  const size_t n3 = size_t(n) * n * n;
  const int nb = grid_for(n3);
  return nb > 256 ? 256 : nb;
}

hipError_t launch_spectrum_bins(int n, double L, const double2* cbuf, int nbins, double* part,
                                double* out3, hipStream_t s) {
  const int nb = spectrum_blocks(n);
  const double n3 = double(n) * n * n;
  hipLaunchKernelGGL(spectrum_bins_kernel, dim3(nb), dim3(kBlock), size_t(3) * nbins * sizeof(double),
                     s, n, cbuf, nbins, 1.0 / (n3 * n3), part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spectrum_finalize_kernel, dim3((nbins + 255) / 256), dim3(256), 0, s, part,
                     nb, nbins, L, out3);
  return hipGetLastError();
}

}  // namespace symlat
