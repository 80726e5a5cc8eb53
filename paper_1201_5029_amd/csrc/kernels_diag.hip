// Observables and state exchange: lattice sums for eq. (2.16), (2.18),
// (2.20), (3.1) at the synchronised state, the constraint solve for p_a, the
// momentum sum S2, and FP64 export/import of the fields.

#include "device.h"

namespace symlat {

namespace {

constexpr int kDiagBlocksMax = 1024;
// target tile count of the 7-point observables pass: two tiles per CU
// (measured at 256^3: 2048 and 1024 tiles took 10 % and 6 % longer; a tile
// writes 2 nsums doubles of partials and the buffer holds 4096 tiles of
// the largest count, the most that n = 1024 makes)
constexpr int kDiagTiles = 512;

struct Bufs {
  const void* phi[2];
  const void* pi[2];
};

Bufs bufs_of(const LatView& v) {
  Bufs B;
  for (int k = 0; k < 2; ++k) {
    B.phi[k] = v.phi[k];
    B.pi[k] = v.pi[k];
  }
  return B;
}

// Per-field sums then the potential: [pi^2, G, phi-s, (phi-s)^2, phi D phi] * NF, V
template <int NF>
constexpr int nsums() { return 5 * NF + 1; }

// G[f] and D[f] of eq. (2.7)-(2.8) at one site with the general cubic
// stencil: the 26 neighbours weighted by class (face, edge, corner).
template <typename T>
__device__ void stencil27_at(const T* __restrict__ phi, const T* __restrict__ pi, double c,
                             double offp, int i, int zs, int n, int x, int y, int z, double f,
                             const Stencil& st, double& D, double& G) {
  const size_t n2 = size_t(n) * n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = z + dz < 0 ? n - 1 : (z + dz >= n ? 0 : z + dz);
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = y + dy < 0 ? n - 1 : (y + dy >= n ? 0 : y + dy);
      for (int dx = -1; dx <= 1; ++dx) {
        const int cls = (dz != 0) + (dy != 0) + (dx != 0);
        if (cls == 0) continue;
        const int xx = x + dx < 0 ? n - 1 : (x + dx >= n ? 0 : x + dx);
        const size_t e = (size_t(zz) * zs + i) * n2 + size_t(yy) * n + xx;
        const double v = offp + fma(c, double(pi[e]), double(phi[e]));
        acc[cls] += v;
        const double d = v - f;
        g[cls] += d * d;
      }
    }
  }
  D = st.c[0] * f + st.c[1] * acc[1] + st.c[2] * acc[2] + st.c[3] * acc[3];
  G = 0.5 * (st.c[1] * g[1] + st.c[2] * g[2] + st.c[3] * g[3]);
}

template <typename T, int NF, int KIND>
__global__ __launch_bounds__(kBlock) void energies_kernel(Bufs B, const DevScalars* sc,
                                                         PotArgs prm, int n, int zs, Stencil st,
                                                         double* partials) {
  constexpr int NV = nsums<NF>();
  __shared__ KSum scratch[4 * NV];
  const int par = sc->parity;
  const T* __restrict__ phi = static_cast<const T*>(B.phi[par]);
  const T* __restrict__ pi = static_cast<const T*>(B.pi[par]);
  const double c = sc->c_pend;
  PotT<double> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = prm.p[i];
  const size_t n2 = size_t(n) * n, n3 = n2 * n;
  // offsets of the stored remainders (0 in FP64 storage), drifted by c
  double offp[NF], offq[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    offq[i] = sc->off_pi[i];
    offp[i] = sc->off_phi[i] + c * offq[i];
  }

  // field i of plane z starts at (z zs + i) n^2
  double shift[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) shift[i] = offp[i] + fma(c, double(pi[i * n2]), double(phi[i * n2]));

  KSum acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = KSum{0.0, 0.0};

  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n3; e += stride) {
    const int x = int(e % n);
    const int y = int((e / n) % n);
    const int z = int(e / n2);
    const size_t r = e - size_t(z) * n2;  // y n + x
    const size_t zm = size_t(z == 0 ? n - 1 : z - 1), zp = size_t(z == n - 1 ? 0 : z + 1);
    // neighbours as (plane, in-plane index)
    const size_t nz[6] = {size_t(z), size_t(z), size_t(z), size_t(z), zm, zp};
    const size_t nr[6] = {r - x + (x == 0 ? n - 1 : x - 1), r - x + (x == n - 1 ? 0 : x + 1),
                          r + (size_t((y == 0 ? n - 1 : y - 1)) - y) * n,
                          r + (size_t((y == n - 1 ? 0 : y + 1)) - y) * n, r, r};
    double f[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const size_t o = (size_t(z) * zs + i) * n2 + r;
      const double pr = double(pi[o]);
      const double pc = offq[i] + pr;
      const double fcv = offp[i] + fma(c, pr, double(phi[o]));
      f[i] = fcv;
      double D, G;
      if (st.kind == 0) {
        double nb[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const size_t on = (nz[q] * zs + i) * n2 + nr[q];
          nb[q] = offp[i] + fma(c, double(pi[on]), double(phi[on]));
        }
        D = -6.0 * fcv;
        G = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          D += nb[q];
          const double d = nb[q] - fcv;
          G += d * d;
        }
        G = 0.5 * G;
      } else {
        stencil27_at<T>(phi, pi, c, offp[i], i, zs, n, x, y, z, fcv, st, D, G);
      }
      kadd(acc[5 * i + 0], pc * pc);
      kadd(acc[5 * i + 1], G);
      const double ds = fcv - shift[i];
      kadd(acc[5 * i + 2], ds);
      kadd(acc[5 * i + 3], ds * ds);
      kadd(acc[5 * i + 4], fcv * D);
    }
    double V, dV[NF];
    potential<KIND, NF, double>(f, pot, V, dV);
    kadd(acc[5 * NF], V);
  }
  block_reduce<NV>(acc, scratch);
  if (threadIdx.x == 0) {
    double* out = partials + size_t(blockIdx.x) * 2 * NV;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      out[2 * k] = acc[k].s;
      out[2 * k + 1] = acc[k].c;
    }
  }
}

// The same sums for the 7-point stencil, walked like the fused pass: a
// workgroup owns a kEX x kEY column tile (one wavefront per row) and marches
// tz planes up in z.  Each lane keeps the drifted field of its site at z-1,
// z, z+1 in registers; plane z goes to LDS (double-buffered, one barrier per
// plane) with a one-cell periodic ring of halo cells that designated lanes
// load, so every plane of the tile is read from memory once.  The loads run
// one plane ahead of the arithmetic (own column two planes ahead, halo one).
// Per site the terms and their order are those of energies_kernel; a lane
// adds its sites' terms plainly over the chunk (at most tz of each) and the
// lanes' and tiles' totals are combined with compensation.
constexpr int kEX = 64, kEY = kBlock / kEX;
constexpr int kELX = kEX + 2, kEPlane = kELX * (kEY + 2);

template <typename T, int NF, int KIND>
__global__ __launch_bounds__(kBlock) void energies7_kernel(Bufs B, const DevScalars* sc,
                                                          PotArgs prm, int n, int zs, int tz,
                                                          double* partials) {
  constexpr int NV = nsums<NF>();
  __shared__ KSum scratch[4 * NV];
  __shared__ double lds[2][NF][kEPlane];
  const int par = sc->parity;
  const T* __restrict__ phi = static_cast<const T*>(B.phi[par]);
  const T* __restrict__ pi = static_cast<const T*>(B.pi[par]);
  const double c = sc->c_pend;
  PotT<double> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = prm.p[i];
  const size_t n2 = size_t(n) * n;
  // offsets of the stored remainders (0 in FP64 storage), drifted by c
  double offp[NF], offq[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    offq[i] = sc->off_pi[i];
    offp[i] = sc->off_phi[i] + c * offq[i];
  }
  double shift[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) shift[i] = offp[i] + fma(c, double(pi[i * n2]), double(phi[i * n2]));

  const int ntx = (n + kEX - 1) / kEX, nty = (n + kEY - 1) / kEY;
  int b = blockIdx.x;
  const int xt = b % ntx;
  b /= ntx;
  const int yt = b % nty;
  const int zt = b / nty;
  const int x0 = xt * kEX, y0 = yt * kEY, z0 = zt * tz;
  const int wx = min(kEX, n - x0), wy = min(kEY, n - y0), zend = min(z0 + tz, n);
  const int tid = int(threadIdx.x), tx = tid % kEX, ty = tid / kEX;
  const bool active = tx < wx && ty < wy;
  const int own = (ty + 1) * kELX + tx + 1;
  // every lane issues the same loads (idle lanes read the tile's first
  // column, in range and unused), so that no branch around them makes the
  // compiler wait for the loads in flight
  const size_t r = active ? size_t(y0 + ty) * n + (x0 + tx) : size_t(y0) * n + x0;

  // halo job: the rows above and below, the columns left and right
  bool hjob = false;
  int hl = 0;
  size_t hr = r;
  if (tid < kEX) {
    if (tid < wx) { hjob = true; hr = size_t((y0 - 1 + n) % n) * n + x0 + tid; hl = tid + 1; }
  } else if (tid < 2 * kEX) {
    const int t = tid - kEX;
    if (t < wx) {
      hjob = true;
      hr = size_t((y0 + wy) % n) * n + x0 + t;
      hl = (wy + 1) * kELX + t + 1;
    }
  } else if (tid < 2 * kEX + kEY) {
    const int q = tid - 2 * kEX;
    if (q < wy) { hjob = true; hr = size_t(y0 + q) * n + (x0 - 1 + n) % n; hl = (q + 1) * kELX; }
  } else if (tid < 2 * kEX + 2 * kEY) {
    const int q = tid - 2 * kEX - kEY;
    if (q < wy) {
      hjob = true;
      hr = size_t(y0 + q) * n + (x0 + wx) % n;
      hl = (q + 1) * kELX + wx + 1;
    }
  }

  auto wrapz = [n](int zz) { return zz < 0 ? zz + n : (zz >= n ? zz - n : zz); };
  // remainders of phi and pi at one site
  auto load = [&](int zz, int i, size_t rr, double& p) {
    const size_t o = (size_t(zz) * zs + i) * n2 + rr;
    p = double(pi[o]);
    return double(phi[o]);
  };

  double part[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) part[k] = 0.0;
  // drifted field at z-1, z, z+1 and momenta at z, z+1 of the own site;
  // drifted halo cell of plane z
  double fm[NF], fc[NF], fp[NF], pc[NF], pp[NF], hc[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    double p = 0.0;
    const double f = load(wrapz(z0 - 1), i, r, p);
    fm[i] = offp[i] + fma(c, p, f);
    const double g = load(z0, i, r, pc[i]);
    fc[i] = offp[i] + fma(c, pc[i], g);
    pc[i] = offq[i] + pc[i];
    const double h = load(wrapz(z0 + 1), i, r, pp[i]);
    fp[i] = offp[i] + fma(c, pp[i], h);
    pp[i] = offq[i] + pp[i];
    const double hh = load(z0, i, hr, p);
    hc[i] = offp[i] + fma(c, p, hh);
  }
  int buf = 0;
  for (int z = z0; z < zend; ++z) {
    // next iteration's loads; past the chunk end they re-read the last
    // plane they need (in range, unused)
    double fn[NF], pn[NF], hn[NF], hq[NF];
    const int z1 = min(z + 1, zend - 1), z2 = wrapz(min(z + 2, zend));
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      fn[i] = load(z2, i, r, pn[i]);
      hn[i] = load(z1, i, hr, hq[i]);
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      if (active) lds[buf][i][own] = fc[i];
      if (hjob) lds[buf][i][hl] = hc[i];
    }
    __syncthreads();
    if (active) {
      double f[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const double* L = lds[buf][i];
        const double fcv = fc[i];
        // neighbours in the order x-1, x+1, y-1, y+1, z-1, z+1
        const double nb[6] = {L[own - 1], L[own + 1], L[own - kELX], L[own + kELX], fm[i], fp[i]};
        double D = -6.0 * fcv, G = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          D += nb[q];
          const double d = nb[q] - fcv;
          G += d * d;
        }
        G = 0.5 * G;
        part[5 * i + 0] += pc[i] * pc[i];
        part[5 * i + 1] += G;
        const double ds = fcv - shift[i];
        part[5 * i + 2] += ds;
        part[5 * i + 3] += ds * ds;
        part[5 * i + 4] += fcv * D;
        f[i] = fcv;
      }
      double V, dV[NF];
      potential<KIND, NF, double>(f, pot, V, dV);
      part[5 * NF] += V;
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      fm[i] = fc[i];
      fc[i] = fp[i];
      pc[i] = pp[i];
      fp[i] = offp[i] + fma(c, pn[i], fn[i]);
      pp[i] = offq[i] + pn[i];
      hc[i] = offp[i] + fma(c, hq[i], hn[i]);
    }
    buf ^= 1;
  }
  KSum acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    acc[k] = KSum{0.0, 0.0};
    kadd(acc[k], part[k]);
  }
  block_reduce<NV>(acc, scratch);
  if (threadIdx.x == 0) {
    double* out = partials + size_t(blockIdx.x) * 2 * NV;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      out[2 * k] = acc[k].s;
      out[2 * k + 1] = acc[k].c;
    }
  }
}

// Reduce energies partials, compute observables; mode 1 also solves the
// constraint H = 0 for p_a (expanding branch) and sets S2.
template <int NF>
__global__ __launch_bounds__(kBlock) void energies_finalize(const double* partials, int nblocks,
                                                           DevScalars* sc, BgConsts K, int n,
                                                           Bufs B, int prec, double* sums_out,
                                                           sl_energies_t* out, int mode) {
  constexpr int NV = nsums<NF>();
  __shared__ KSum scratch[4 * NV];
  KSum v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = KSum{0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    const double* p = partials + size_t(b) * 2 * NV;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = kcombine(v[k], KSum{p[2 * k], p[2 * k + 1]});
  }
  block_reduce<NV>(v, scratch);
  if (threadIdx.x != 0) return;
  DevScalars S = *sc;
  double s[NV];
  for (int k = 0; k < NV; ++k) {
    s[k] = v[k].s + v[k].c;
    sums_out[k] = s[k];
  }
  const size_t n2 = size_t(n) * n;
  const double VL = K.VL;
  const double a = S.a;
  const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
  sl_energies_t E;
  for (int i = 0; i < 8; ++i) E.kin[i] = E.grad[i] = E.mean[i] = E.var[i] = 0.0;
  double S2 = 0.0, SdD = 0.0, skin = 0.0, sgrad = 0.0;
  const int par = S.parity;
  for (int i = 0; i < NF; ++i) {
    // shift used by the sum kernel: phi_sync at site 0
    double sh;
    const double offp = S.off_phi[i] + S.c_pend * S.off_pi[i];
    if (prec == SL_FP32) {
      const float* ph = static_cast<const float*>(B.phi[par]);
      const float* pp = static_cast<const float*>(B.pi[par]);
      sh = offp + fma(S.c_pend, double(pp[i * n2]), double(ph[i * n2]));
    } else {
      const double* ph = static_cast<const double*>(B.phi[par]);
      const double* pp = static_cast<const double*>(B.pi[par]);
      sh = offp + fma(S.c_pend, pp[i * n2], ph[i * n2]);
    }
    E.kin[i] = (s[5 * i] / VL) / (2.0 * a6);
    E.grad[i] = (s[5 * i + 1] / VL) / (2.0 * a2 * K.dx2);
    const double m1 = s[5 * i + 2] / VL;
    E.mean[i] = sh + m1;
    E.var[i] = s[5 * i + 3] / VL - m1 * m1;
    S2 += s[5 * i];
    SdD += s[5 * i + 4];
    skin += E.kin[i];
    sgrad += E.grad[i];
  }
  const double SV = s[5 * NF];
  E.pot = SV / VL;
  E.rho = skin + sgrad + E.pot;
  E.pressure = skin - sgrad / 3.0 - E.pot;
  E.w_eos = E.rho != 0.0 ? E.pressure / E.rho : __builtin_nan("");
  // field part of eq. (2.20) plus the radiation and matter terms
  const double Hf = S2 / (2.0 * a2) - a2 * SdD / (2.0 * K.dx2) + a4 * SV;
  const double Hext = K.VL_rho_r + a * K.VL_rho_m;
  if (mode == 1) {
    S.S2 = S2;
    if (K.expand) {
      const double E0 = Hf + Hext;
      if (E0 >= 0.0) {
        S.p_a = -sqrt(12.0 * VL * K.mpl2 * E0);
      } else {
        S.p_a = __builtin_nan("");
        S.status |= kStatusNonFinite;
      }
    } else {
      S.p_a = 0.0;
    }
    *sc = S;
  }
  E.eta = S.eta;
  E.a = a;
  E.p_a = S.p_a;
  if (K.expand) {
    E.hubble = -S.p_a / (6.0 * VL * K.mpl2 * a2);
    const double rho_tot = E.rho + (K.VL_rho_r / VL) / a4 + (K.VL_rho_m / VL) / (a2 * a);
    E.friedmann_residual = fabs(rho_tot / (3.0 * K.mpl2 * E.hubble * E.hubble) - 1.0);
    E.h_total = -S.p_a * S.p_a / (12.0 * VL * K.mpl2) + Hf + Hext;
  } else {
    E.hubble = 0.0;
    E.friedmann_residual = __builtin_nan("");
    E.h_total = Hf + Hext;
  }
  *out = E;
}

template <typename T, int NF, int KIND>
hipError_t energies_t(const LatView& v, double* sums, sl_energies_t* out, int mode, hipStream_t s) {
  const Bufs B = bufs_of(v);
  const size_t n3 = size_t(v.n) * v.n * v.n;
  int nb = 0;
  if (v.st.kind == 0) {
    // z-chunks so that the tiles number about kDiagTiles (at most one chunk
    // per plane)
    const int cols = ((v.n + kEX - 1) / kEX) * ((v.n + kEY - 1) / kEY);
    int ntz = kDiagTiles / cols;
    ntz = ntz < 1 ? 1 : (ntz > v.n ? v.n : ntz);
    const int tz = (v.n + ntz - 1) / ntz;
    nb = cols * ((v.n + tz - 1) / tz);
    hipLaunchKernelGGL((energies7_kernel<T, NF, KIND>), dim3(nb), dim3(kBlock), 0, s, B, v.sc,
                       v.prm, v.n, v.zs, tz, v.partials);
  } else {
    nb = int((n3 + kBlock - 1) / kBlock);
    if (nb > kDiagBlocksMax) nb = kDiagBlocksMax;
    hipLaunchKernelGGL((energies_kernel<T, NF, KIND>), dim3(nb), dim3(kBlock), 0, s, B, v.sc,
                       v.prm, v.n, v.zs, v.st, v.partials);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((energies_finalize<NF>), dim3(1), dim3(kBlock), 0, s, v.partials, nb, v.sc,
                     v.bg, v.n, B, v.prec, sums, out, mode);
  return hipGetLastError();
}

template <typename T>
hipError_t energies_dispatch(const LatView& v, double* sums, sl_energies_t* out, int mode,
                             hipStream_t s) {
  switch (v.pot) {
    case SL_POT_CHAOTIC2: return energies_t<T, 2, SL_POT_CHAOTIC2>(v, sums, out, mode, s);
    case SL_POT_OSCILLON: return energies_t<T, 1, SL_POT_OSCILLON>(v, sums, out, mode, s);
    case SL_POT_QBALL_LOG: return energies_t<T, 2, SL_POT_QBALL_LOG>(v, sums, out, mode, s);
    default: break;
  }
  switch (v.nf) {
    case 1: return energies_t<T, 1, SL_POT_FREE>(v, sums, out, mode, s);
    case 2: return energies_t<T, 2, SL_POT_FREE>(v, sums, out, mode, s);
    case 3: return energies_t<T, 3, SL_POT_FREE>(v, sums, out, mode, s);
    case 4: return energies_t<T, 4, SL_POT_FREE>(v, sums, out, mode, s);
    case 5: return energies_t<T, 5, SL_POT_FREE>(v, sums, out, mode, s);
    case 6: return energies_t<T, 6, SL_POT_FREE>(v, sums, out, mode, s);
    case 7: return energies_t<T, 7, SL_POT_FREE>(v, sums, out, mode, s);
    case 8: return energies_t<T, 8, SL_POT_FREE>(v, sums, out, mode, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void sum_pi2_kernel(Bufs B, const DevScalars* sc,
                                                        size_t count, size_t n3, size_t n2, int zs,
                                                        double* partials) {
  __shared__ KSum scratch[4];
  const T* __restrict__ pi = static_cast<const T*>(B.pi[sc->parity]);
  KSum acc[1] = {{0.0, 0.0}};
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += stride) {
    const size_t i = e / n3;  // field i, site e - i n^3
    const double p = sc->off_pi[i] + double(pi[field_site(int(i), e - i * n3, zs, n2)]);
    kadd(acc[0], p * p);
  }
  block_reduce<1>(acc, scratch);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = acc[0].s;
    partials[2 * blockIdx.x + 1] = acc[0].c;
  }
}

__global__ __launch_bounds__(kBlock) void sum_pi2_finalize(const double* partials, int nblocks,
                                                          DevScalars* sc) {
  __shared__ KSum scratch[4];
  KSum v[1] = {{0.0, 0.0}};
  for (int b = threadIdx.x; b < nblocks; b += kBlock)
    v[0] = kcombine(v[0], KSum{partials[2 * b], partials[2 * b + 1]});
  block_reduce<1>(v, scratch);
  if (threadIdx.x == 0) {
    const double S2 = v[0].s + v[0].c;
    sc->S2 = S2;
    if (!dev_finite(S2)) sc->status |= kStatusNonFinite;
  }
}

// Device offset of host element e: the host arrays are [field][z][y][x].
__device__ __forceinline__ size_t device_index(size_t e, int zs, size_t n2, size_t n3) {
  const size_t i = e / n3;
  return field_site(int(i), e - i * n3, zs, n2);
}

template <typename T>
__global__ void export_kernel(Bufs B, const DevScalars* sc, size_t count, int nf, int zs,
                              size_t n2, double* phi_out, double* pi_out) {
  const int par = sc->parity;
  const T* __restrict__ phi = static_cast<const T*>(B.phi[par]);
  const T* __restrict__ pi = static_cast<const T*>(B.pi[par]);
  const double c = sc->c_pend;
  const size_t n3 = count / nf;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += stride) {
    const size_t d = device_index(e, zs, n2, n3);
    const size_t i = e / n3;
    const double pr = double(pi[d]);
    if (phi_out) phi_out[e] = (sc->off_phi[i] + c * sc->off_pi[i]) + fma(c, pr, double(phi[d]));
    if (pi_out) pi_out[e] = sc->off_pi[i] + pr;
  }
}

template <typename T>
__global__ void import_kernel(void* phi0, void* pi0, size_t count, int nf, int zs, size_t n2,
                              const double* phi_in, const double* pi_in, Offsets off) {
  T* __restrict__ phi = static_cast<T*>(phi0);
  T* __restrict__ pi = static_cast<T*>(pi0);
  const size_t n3 = count / nf;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += stride) {
    const size_t d = device_index(e, zs, n2, n3);
    const size_t i = e / n3;
    phi[d] = static_cast<T>(phi_in[e] - off.phi[i]);
    pi[d] = static_cast<T>(pi_in[e] - off.pi[i]);
  }
}

// One record per batch member, in table order, for a single read-back.
__global__ void gather_scalars_kernel(const BatchRun* __restrict__ runs, int nruns,
                                      DevScalars* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nruns) out[r] = *runs[r].sc[0];
}

__global__ void reset_scalars_kernel(DevScalars* sc, double a, double p_a, Offsets off) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    DevScalars S = *sc;  // keeps the history buffer; a reset restarts it
    for (int i = 0; i < kMaxFields; ++i) {
      S.off_phi[i] = off.phi[i];
      S.off_pi[i] = off.pi[i];
    }
    S.a = a;
    S.p_a = p_a;
    S.eta = 0.0;
    S.S2 = 0.0;
    S.c_pend = 0.0;
    S.c_next = 0.0;
    S.alpha = 0.0;
    S.beta = 0.0;
    S.a_kick = a;
    S.S3_last = 0.0;
    S.parity = 0;
    S.status = 0;
    S.hist_n = 0;
    *sc = S;
  }
}

int grid_for(size_t count) {
  size_t nb = (count + kBlock - 1) / kBlock;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  return int(nb);
}

}  // namespace

hipError_t launch_energies(const LatView& v, double* sums, sl_energies_t* out, int mode,
                           hipStream_t s) {
  return v.prec == SL_FP32 ? energies_dispatch<float>(v, sums, out, mode, s)
                           : energies_dispatch<double>(v, sums, out, mode, s);
}

hipError_t launch_sum_pi2(const LatView& v, hipStream_t s) {
  const size_t count = size_t(v.nf) * v.n * v.n * v.n;
  const int nb = grid_for(count) > kDiagBlocksMax ? kDiagBlocksMax : grid_for(count);
  const Bufs B = bufs_of(v);
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(sum_pi2_kernel<float>, dim3(nb), dim3(kBlock), 0, s, B, v.sc, count,
                       count / v.nf, size_t(v.n) * v.n, v.zs, v.partials);
  else
    hipLaunchKernelGGL(sum_pi2_kernel<double>, dim3(nb), dim3(kBlock), 0, s, B, v.sc, count,
                       count / v.nf, size_t(v.n) * v.n, v.zs, v.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_pi2_finalize, dim3(1), dim3(kBlock), 0, s, v.partials, nb, v.sc);
  return hipGetLastError();
}

hipError_t launch_export(const LatView& v, double* phi_out, double* pi_out, hipStream_t s) {
  const size_t count = size_t(v.nf) * v.n * v.n * v.n;
  const Bufs B = bufs_of(v);
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(export_kernel<float>, dim3(grid_for(count)), dim3(kBlock), 0, s, B, v.sc,
                       count, v.nf, v.zs, size_t(v.n) * v.n, phi_out, pi_out);
  else
    hipLaunchKernelGGL(export_kernel<double>, dim3(grid_for(count)), dim3(kBlock), 0, s, B, v.sc,
                       count, v.nf, v.zs, size_t(v.n) * v.n, phi_out, pi_out);
  return hipGetLastError();
}

hipError_t launch_import(const LatView& v, const double* phi_in, const double* pi_in, double a,
                         double p_a, const Offsets& off, hipStream_t s) {
  const size_t count = size_t(v.nf) * v.n * v.n * v.n;
  if (v.prec == SL_FP32)
    hipLaunchKernelGGL(import_kernel<float>, dim3(grid_for(count)), dim3(kBlock), 0, s, v.phi[0],
                       v.pi[0], count, v.nf, v.zs, size_t(v.n) * v.n, phi_in, pi_in, off);
  else
    hipLaunchKernelGGL(import_kernel<double>, dim3(grid_for(count)), dim3(kBlock), 0, s, v.phi[0],
                       v.pi[0], count, v.nf, v.zs, size_t(v.n) * v.n, phi_in, pi_in, off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reset_scalars_kernel, dim3(1), dim3(64), 0, s, v.sc, a, p_a, off);
  return hipGetLastError();
}

hipError_t launch_gather_scalars(const BatchRun* runs_dev, int nruns, DevScalars* out_dev,
                                 hipStream_t s) {
  if (nruns <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_scalars_kernel, dim3((nruns + 255) / 256), dim3(256), 0, s, runs_dev,
                     nruns, out_dev);
  return hipGetLastError();
}

hipError_t launch_reset_scalars(const LatView& v, double a, double p_a, const Offsets& off,
                                hipStream_t s) {
  hipLaunchKernelGGL(reset_scalars_kernel, dim3(1), dim3(64), 0, s, v.sc, a, p_a, off);
  return hipGetLastError();
}

}  // namespace symlat
