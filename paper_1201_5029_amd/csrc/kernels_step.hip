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
// grid-wide dependency: a stage is one pass plus a scalar update, which the
// next pass runs itself (a chained pass, see Chain) or a small finalize
// kernel runs after it.
//
// Data layout: in phi and pi the fields of each z-plane follow one another
// (x fastest), planes P.zs n^2 elements apart (zs = nf, or 2 nf when phi and
// pi of a parity share one block, interleaved by plane); two ping-pong
// buffers: the pass reads buffer `parity` and writes the other one, so no
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


// VX consecutive x-sites per lane, moved with one vector load/store.
template <typename T, int VX>
struct Vec {
  T v[VX];
};

template <typename T, int VX>
__device__ __forceinline__ Vec<T, VX> ldv(const T* __restrict__ p) {
  Vec<T, VX> r;
  if constexpr (VX == 1) {
    r.v[0] = p[0];
  } else if constexpr (VX == 4 && sizeof(T) == 8) {
    const double4 q = *reinterpret_cast<const double4*>(p);
    r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
  } else if constexpr (VX == 4) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
  } else if constexpr (sizeof(T) == 8) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    r.v[0] = q.x;
    r.v[1] = q.y;
  } else {
    const float2 q = *reinterpret_cast<const float2*>(p);
    r.v[0] = q.x;
    r.v[1] = q.y;
  }
  return r;
}

template <typename T, int VX>
__device__ __forceinline__ void stv(T* __restrict__ p, const T (&v)[VX]) {
  if constexpr (VX == 1) {
    p[0] = v[0];
  } else if constexpr (VX == 4 && sizeof(T) == 8) {
    *reinterpret_cast<double4*>(p) = make_double4(v[0], v[1], v[2], v[3]);
  } else if constexpr (VX == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else if constexpr (sizeof(T) == 8) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  } else {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  }
}

// The same stores with the non-temporal hint: the results of a pass are
// read only by the next pass, so they should not displace the halo rows and
// planes that neighbouring tiles are about to read from the L2.
template <typename T, int VX>
__device__ __forceinline__ void stv_nt(T* __restrict__ p, const T (&v)[VX]) {
  if constexpr (VX == 2 && sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 q = {v[0], v[1]};
    __builtin_nontemporal_store(q, reinterpret_cast<d2*>(p));
  } else if constexpr (VX == 4 && sizeof(T) == 8) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    const d4 q = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(q, reinterpret_cast<d4*>(p));
  } else if constexpr (VX == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 q = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(q, reinterpret_cast<f4*>(p));
  } else if constexpr (VX == 2) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 q = {v[0], v[1]};
    __builtin_nontemporal_store(q, reinterpret_cast<f2*>(p));
  } else {
    __builtin_nontemporal_store(v[0], p);
  }
}

template <bool NT, typename T, int VX>
__device__ __forceinline__ void stv_mode(T* __restrict__ p, const T (&v)[VX]) {
  if constexpr (NT)
    stv_nt<T, VX>(p, v);
  else
    stv<T, VX>(p, v);
}

// Workgroups are dealt to the 8 XCDs round-robin (id mod 8).  Renumber them
// so that each XCD receives a contiguous run of tiles: neighbouring tiles,
// whose halos overlap, then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int kXcd = 8;
  const int per = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd, i = b / kXcd;
  return x * per + (x < rem ? x : rem) + i;
}

// FP32 storage: the offsets of the state this pass writes -- the homogeneous
// parts of the stage's drift and kick, fbar = off_phi + c off_pi and
// pibar = off_pi - beta dV(fbar), in FP64 (every lane forms the same values)
// -- and the constants of the difference form of dV around fbar.  The first
// tile records them for the stage update (finalize or next chained pass).
template <int KIND, int NF, typename T>
__device__ __forceinline__ void split_offsets(const PassParams& P, const DevScalars& S,
                                              double* offs_out, int tile_id, double (&fbar)[NF],
                                              double (&pibar)[NF], T (&fbT)[NF], SplitK<T>& sk) {
  const double c = S.c_next, beta = S.beta;
  PotT<double> pd;
#pragma unroll
  for (int k = 0; k < kMaxFields; ++k) pd.p[k] = P.prm.p[k];
  double V0, dv[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) fbar[i] = fma(c, S.off_pi[i], S.off_phi[i]);
  potential<KIND, NF, double>(fbar, pd, V0, dv);
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    pibar[i] = fma(-beta, dv[i], S.off_pi[i]);
    fbT[i] = static_cast<T>(fbar[i]);
  }
  sk = split_consts<KIND, NF, T>(fbar, P.prm);
  if (tile_id == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      offs_out[i] = fbar[i];
      offs_out[kMaxFields + i] = pibar[i];
    }
  }
}

// The scalars of this stage into S (LDS, every thread of the workgroup sees
// them after the barrier): read from buffer s_in, or, for a chained pass,
// formed by finishing the previous stage (see Chain).  All threads call.
// A chained pass reads the previous stage's records (scalar words, offset
// record, this thread's share of the per-tile partials) at the very start,
// before the loads that depend on the state's parity, so that they are
// first in the memory queue and the stage update overlaps the prologue's
// plane loads.  Up to kChainMaxTiles = 4 x 256 tiles.
struct ChainPre {
  double word;
  double p[4][6];
};
__device__ void chain_prefetch(const PassParams& P, const Chain& C, ChainPre& cp);
template <bool CH>
__device__ void stage_scalars(const PassParams& P, const Chain& C, int tile_id, DevScalars& S,
                              KSum* scratch, bool fresh, const ChainPre& cp);

// PF = 1: the next plane is loaded at the top of each z-iteration and used
// at once.  PF = 2: software pipeline -- the loads for plane z+1 (own column
// one plane further ahead, and the halo) are issued right after the barrier
// of plane z, before plane z's stores.  PF = 3: the same, one plane further
// ahead again, with two register sets used in turn.  Vector-memory counters retire in
// issue order, so a wavefront does not wait for its own stores before it
// uses the next plane's data -- provided every lane issues the same memory
// instructions: idle lanes (past the tile's ragged x or y edge, or past its
// rows) shadow the nearest active lane of the tile -- they load its column,
// compute its sites and store the same values to the same addresses, which
// costs no memory traffic -- but add nothing to the partial sums, and x-halo
// cells are fetched as the aligned VX-wide group that contains them.
template <int I>
struct Half {
  static constexpr int value = I;
};

template <typename T, int NF, int KIND, int VX, int PF, bool NT, bool CH>
__device__ __forceinline__ void pass_tile(const PassParams& P, const Chain& C, int tile_id, T* lds,
                                          KSum* red_scratch, DevScalars& S, bool fresh) {
  ChainPre cp;
  if constexpr (CH)
    if (C.chain && fresh) chain_prefetch(P, C, cp);
  // parity of the state this pass reads (a chained pass flips it when it
  // finishes the previous stage)
  const int par = P.sc[C.s_in]->parity ^ C.chain;
  const T* __restrict__ phi_in = static_cast<const T*>(P.phi[par]);
  const T* __restrict__ pi_in = static_cast<const T*>(P.pi[par]);
  T* __restrict__ phi_out = static_cast<T*>(P.phi_w[par ^ 1]);
  T* __restrict__ pi_out = static_cast<T*>(P.pi_w[par ^ 1]);
  T c = T(0), alpha = T(0), beta = T(0);  // set once the stage scalars are in
  PotT<T> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = static_cast<T>(P.prm.p[i]);
  // FP32 storage: the arrays hold remainders around FP64 offsets; the
  // offsets of the state this pass writes come with the stage coefficients
  constexpr bool kSplit = sizeof(T) == 4;
  double fbar[NF], pibar[NF];
  T fbT[NF];
  SplitK<T> sk{};

  const int n = P.n;
  const size_t n2 = size_t(n) * n;

  // tile of this workgroup (x tiles fastest, then y, then z chunks)
  int b = tile_id;
  const int xt = b % P.ntx;
  b /= P.ntx;
  const int yt = b % P.nty;
  const int zt = b / P.nty;
  const int TW = P.tx * VX;  // tile width in sites
  const int x0 = xt * TW, y0 = yt * P.ty, z0 = zt * P.tz;
  const int wx = min(TW, n - x0), wy = min(P.ty, n - y0), zc = min(P.tz, n - z0);
  const int zend = z0 + zc;  // exclusive; plane zend (mod n) is the upper halo

  const int tid = threadIdx.x;
  const int ty = tid / P.tx;  // lanes past TX*TY (ty = TY) are idle
  const int tx = tid - ty * P.tx;
  const bool active = (tx * VX < wx) && (ty < wy);
  const int LX = TW + 2;
  const int plane = LX * (P.ty + 2);
  // lane whose sites this lane computes: itself, or for an idle lane the
  // active lane at the clamped position
  const int sx = min(tx, wx / VX - 1), sy = min(ty, wy - 1);
  // LDS index of the first own site and the own column
  const int own = (sy + 1) * LX + 1 + sx * VX;
  const size_t col = size_t(y0 + sy) * n + (x0 + sx * VX);

  // halo job: 1 = VX-wide row segment, 2 = left x-halo cell, 3 = right
  // x-halo cell, 0 = none.  Every lane loads one aligned VX-wide group per
  // field and plane (its own column when it has no job).
  int hjob = 0, hl = 0;
  size_t hcol = col;
  {
    const int TX = P.tx, TY = P.ty;
    int hx = -1, hy = 0;
    if (tid < TX) {
      if (tid * VX < wx) { hjob = 1; hx = x0 + tid * VX; hy = (y0 - 1 + n) % n; hl = 1 + tid * VX; }
    } else if (tid < 2 * TX) {
      const int t = tid - TX;
      if (t * VX < wx) { hjob = 1; hx = x0 + t * VX; hy = (y0 + wy) % n; hl = (wy + 1) * LX + 1 + t * VX; }
    } else if (tid < 2 * TX + TY) {
      const int r = tid - 2 * TX;
      // group [x0 - VX, x0) holds the left neighbour x0 - 1 as element VX - 1
      if (r < wy) { hjob = 2; hx = (x0 - VX + n) % n; hy = y0 + r; hl = (r + 1) * LX; }
    } else if (tid < 2 * TX + 2 * TY) {
      const int r = tid - 2 * TX - TY;
      // group [x0 + wx, x0 + wx + VX) holds the right neighbour as element 0
      if (r < wy) { hjob = 3; hx = (x0 + wx) % n; hy = y0 + r; hl = (r + 1) * LX + wx + 1; }
    }
    if (hx >= 0) hcol = size_t(hy) * n + hx;
  }

  auto wrap = [n](int z) { return z >= n ? z - n : z; };

  KSum acc_dd{0.0, 0.0}, acc_v{0.0, 0.0}, acc_p{0.0, 0.0};
  // drifted field at z-1, z, z+1 and momenta at z, z+1 of the own sites
  T fm[NF][VX], fc[NF][VX], fp[NF][VX], pc[NF][VX], pp[NF][VX];
  // raw loads in flight: own column and halo
  T nph[NF][VX], npi[NF][VX], hph[NF][VX], hpi[NF][VX];

  auto load_own_into = [&](int zz, T (&oph)[NF][VX], T (&opi)[NF][VX]) {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const size_t o = (size_t(zz) * P.zs + i) * n2 + col;
      const Vec<T, VX> u = ldv<T, VX>(phi_in + o), w = ldv<T, VX>(pi_in + o);
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        oph[i][v] = u.v[v];
        opi[i][v] = w.v[v];
      }
    }
  };
  auto load_own = [&](int zz) { load_own_into(zz, nph, npi); };
  auto load_halo_into = [&](int zz, T (&oph)[NF][VX], T (&opi)[NF][VX]) {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const size_t o = (size_t(zz) * P.zs + i) * n2 + hcol;
      const Vec<T, VX> u = ldv<T, VX>(phi_in + o), w = ldv<T, VX>(pi_in + o);
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        oph[i][v] = u.v[v];
        opi[i][v] = w.v[v];
      }
    }
  };
  auto load_halo = [&](int zz) { load_halo_into(zz, hph, hpi); };
  auto halo_to_lds_from = [&](T* L, const T (&gph)[NF][VX], const T (&gpi)[NF][VX]) {
    if (hjob == 1) {
#pragma unroll
      for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int v = 0; v < VX; ++v) L[i * plane + hl + v] = drift(gph[i][v], gpi[i][v], c);
    } else if (hjob >= 2) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const T f = hjob == 2 ? gph[i][VX - 1] : gph[i][0];
        const T q = hjob == 2 ? gpi[i][VX - 1] : gpi[i][0];
        L[i * plane + hl] = drift(f, q, c);
      }
    }
  };
  auto halo_to_lds = [&](T* L) { halo_to_lds_from(L, hph, hpi); };
  // fp, pp from raw own-column loads
  auto take_from = [&](const T (&oph)[NF][VX], const T (&opi)[NF][VX]) {
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        pp[i][v] = opi[i][v];
        fp[i][v] = drift(oph[i][v], opi[i][v], c);
      }
  };
  auto take_next = [&]() { take_from(nph, npi); };

  // prologue: planes z0 - 1 and z0 of the own column (and for PF = 2 the
  // first iteration's loads: own plane z0 + 1, halo of plane z0), all
  // issued before the stage scalars are formed, so that their latency
  // overlaps the scalar update
  T mph[NF][VX], mpi[NF][VX], cph[NF][VX], cpi[NF][VX];
  // second register set of the depth-3 pipeline (the first: nph/npi, hph/hpi)
  [[maybe_unused]] T qph[NF][VX], qpi[NF][VX], gph[NF][VX], gpi[NF][VX];
  load_own_into((z0 - 1 + n) % n, mph, mpi);
  load_own_into(z0, cph, cpi);
  if constexpr (PF == 2) {
    load_own(wrap(z0 + 1));
    load_halo(z0);
  }
  if constexpr (PF == 3) {
    // planes z0 + 1 and z0 + 2 of the own column and the halo of z0 and
    // z0 + 1, each pair followed by 2 NF stores into the sink slot: the same
    // trailing sequence as two loop iterations (see the PF = 2 sink below)
    T* sink = static_cast<T*>(P.sink) + size_t(tid) * (2 * NF * VX);
    T zero[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) zero[v] = T(0);
    load_own(wrap(min(z0 + 1, zend)));
    load_halo(z0);
#pragma unroll
    for (int i = 0; i < 2 * NF; ++i) stv<T, VX>(sink + i * VX, zero);
    load_own_into(wrap(min(z0 + 2, zend)), qph, qpi);
    load_halo_into(min(z0 + 1, zend - 1), gph, gpi);
#pragma unroll
    for (int i = 0; i < 2 * NF; ++i) stv<T, VX>(sink + i * VX, zero);
  }
  stage_scalars<CH>(P, C, tile_id, S, red_scratch, fresh, cp);
  c = static_cast<T>(S.c_next);
  alpha = static_cast<T>(S.alpha);
  beta = static_cast<T>(S.beta);
  if constexpr (kSplit) split_offsets<KIND, NF, T>(P, S, P.offs[C.p_out], tile_id, fbar, pibar, fbT, sk);
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int v = 0; v < VX; ++v) fm[i][v] = drift(mph[i][v], mpi[i][v], c);
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int v = 0; v < VX; ++v) {
      pc[i][v] = cpi[i][v];
      fc[i][v] = drift(cph[i][v], cpi[i][v], c);
    }
  if constexpr (PF == 2) {
    // Same trailing sequence as a loop iteration (loads, then 2 NF stores),
    // so the wait counts the compiler derives at the loop head do not cover
    // the previous plane's stores.  The stores go to a per-thread sink slot
    // (cached stores: every workgroup reuses the same slots).
    T* sink = static_cast<T*>(P.sink) + size_t(tid) * (2 * NF * VX);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      stv<T, VX>(sink + (2 * i) * VX, fc[i]);
      stv<T, VX>(sink + (2 * i + 1) * VX, pc[i]);
    }
  }

  // the update of plane z from the drifted plane in LDS: kick, sums, the
  // stores of plane z, and the shift of the register planes
  auto update_plane = [&](int z, const T* L) {
    double dd = 0.0, p2 = 0.0, vs = 0.0;
    T pn[NF][VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
      T f[NF], D[NF], dV[NF], V;
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const T* Li = L + i * plane + own + v;
        f[i] = fc[i][v];
        D[i] = ((Li[-1] + Li[1]) + (Li[-LX] + Li[LX])) + (fm[i][v] + fp[i][v]) - T(6) * f[i];
      }
      if constexpr (kSplit)
        potential_split<KIND, NF, T>(fbT, f, pot, sk, V, dV);  // dV(fbar + f) - dV(fbar)
      else
        potential<KIND, NF, T>(f, pot, V, dV);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        pn[i][v] = pc[i][v] + alpha * D[i] - beta * dV[i];
        if constexpr (kSplit) {
          dd += (fbar[i] + double(f[i])) * double(D[i]);
          const double q = pibar[i] + double(pn[i][v]);
          p2 += q * q;
        } else {
          dd += double(f[i]) * double(D[i]);
          p2 += double(pn[i][v]) * double(pn[i][v]);
        }
      }
      vs += double(V);
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const size_t oc = (size_t(z) * P.zs + i) * n2 + col;
      stv_mode<NT, T, VX>(phi_out + oc, fc[i]);
      stv_mode<NT, T, VX>(pi_out + oc, pn[i]);
    }
    if (active) {
      kadd(acc_dd, dd);
      kadd(acc_v, vs);
      kadd(acc_p, p2);
    }
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        fm[i][v] = fc[i][v];
        fc[i][v] = fp[i][v];
        pc[i][v] = pp[i][v];
      }
  };

  if constexpr (PF != 3) {
    int buf = 0;
    for (int z = z0; z < zend; ++z) {
      T* L = lds + size_t(buf) * NF * plane;
      if constexpr (PF == 1) {
        load_own(wrap(z + 1));
        take_next();
        load_halo(z);
      } else {
        take_next();  // loads issued before the previous plane's stores
      }
      halo_to_lds(L);
      if (active) {
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
          for (int v = 0; v < VX; ++v) L[i * plane + own + v] = fc[i][v];
      }
      __syncthreads();
      if constexpr (PF == 2) {
        // next plane's loads go out before this plane's stores; past the end
        // of the chunk they re-read the last plane (in range, unused)
        load_own(wrap(min(z + 2, zend)));
        load_halo(min(z + 1, zend - 1));
      }
      update_plane(z, L);
      buf ^= 1;
    }
  } else {
    // Depth 3: after the barrier of plane z the loads of own plane z + 3 and
    // of the halo of plane z + 2 go out, into the register set that plane z
    // has just emptied (set (z - z0) & 1, as is the LDS buffer).  Planes go
    // in pairs so that each half names its set at compile time; past the end
    // of the chunk the loads re-read the last planes (in range, unused).
    auto half = [&](auto h, int z) {
      constexpr int H = decltype(h)::value;
      T* L = lds + size_t(H) * NF * plane;
      if constexpr (H == 0) {
        take_from(nph, npi);
        halo_to_lds_from(L, hph, hpi);
      } else {
        take_from(qph, qpi);
        halo_to_lds_from(L, gph, gpi);
      }
      if (active) {
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
          for (int v = 0; v < VX; ++v) L[i * plane + own + v] = fc[i][v];
      }
      __syncthreads();
      if constexpr (H == 0) {
        load_own_into(wrap(min(z + 3, zend)), nph, npi);
        load_halo_into(min(z + 2, zend - 1), hph, hpi);
      } else {
        load_own_into(wrap(min(z + 3, zend)), qph, qpi);
        load_halo_into(min(z + 2, zend - 1), gph, gpi);
      }
      update_plane(z, L);
    };
    int z = z0;
    for (; z + 1 < zend; z += 2) {
      half(Half<0>{}, z);
      half(Half<1>{}, z + 1);
    }
    if (z < zend) half(Half<0>{}, z);
  }

  KSum v3[3] = {acc_dd, acc_v, acc_p};
  block_reduce<3>(v3, red_scratch);
  if (threadIdx.x == 0) {
    double* out = P.partials[C.p_out] + size_t(tile_id) * 6;
    out[0] = v3[0].s; out[1] = v3[0].c;
    out[2] = v3[1].s; out[3] = v3[1].c;
    out[4] = v3[2].s; out[5] = v3[2].c;
  }
}

// The same stage pass with any member of the cubic stencil family of
// eq. (2.7): D = c0 f + c1 (6 faces) + c2 (12 edges) + c3 (8 corners).  Per
// plane p of the own sites the lane forms, from the drifted plane in LDS
// (halo ring including the four corner cells), the centre value f(p), the
// in-plane face sum F(p) = f(x+-1) + f(y+-1) and the in-plane corner sum
// C(p) = f(x+-1, y+-1).  Then, for the site at plane z,
//   faces = F(z) + f(z-1) + f(z+1),  edges = C(z) + F(z-1) + F(z+1),
//   corners = C(z-1) + C(z+1),
// so a ring of three (f, F, C) triples in registers replaces a second LDS
// plane.  The ring lags the loads by one plane: the chunk walks planes
// z0 - 1 .. zend and writes plane p - 1 while plane p is in LDS.  VX
// consecutive sites per lane (one vector load/store); the memory
// instructions are uniform across lanes (idle lanes load the tile's first
// column and store into the sink; x-halo and corner cells are fetched as the
// aligned VX-wide group that contains them), and the loads of plane p + 1 go
// out after the barrier, before the stores of plane p - 1.  NT: the results
// (and the idle lanes' sink stores) are written with non-temporal stores.
template <typename T, int NF, int KIND, int VX, bool NT, bool CH>
__device__ __forceinline__ void pass_tile27(const PassParams& P, const Chain& C, int tile_id, T* lds,
                                            KSum* red_scratch, DevScalars& S, bool fresh) {
  ChainPre cp;
  if constexpr (CH)
    if (C.chain && fresh) chain_prefetch(P, C, cp);
  const int par = P.sc[C.s_in]->parity ^ C.chain;
  const T* __restrict__ phi_in = static_cast<const T*>(P.phi[par]);
  const T* __restrict__ pi_in = static_cast<const T*>(P.pi[par]);
  T* __restrict__ phi_out = static_cast<T*>(P.phi_w[par ^ 1]);
  T* __restrict__ pi_out = static_cast<T*>(P.pi_w[par ^ 1]);
  T c = T(0), alpha = T(0), beta = T(0);  // set once the stage scalars are in
  const T w0 = static_cast<T>(P.stc[0]), w1 = static_cast<T>(P.stc[1]);
  const T w2 = static_cast<T>(P.stc[2]), w3 = static_cast<T>(P.stc[3]);
  PotT<T> pot;
#pragma unroll
  for (int i = 0; i < kMaxFields; ++i) pot.p[i] = static_cast<T>(P.prm.p[i]);
  constexpr bool kSplit = sizeof(T) == 4;  // remainders around FP64 offsets
  double fbar[NF], pibar[NF];
  T fbT[NF];
  SplitK<T> sk{};

  const int n = P.n;
  const size_t n2 = size_t(n) * n;

  int b = tile_id;
  const int xt = b % P.ntx;
  b /= P.ntx;
  const int yt = b % P.nty;
  const int zt = b / P.nty;
  const int TW = P.tx * VX;
  const int x0 = xt * TW, y0 = yt * P.ty, z0 = zt * P.tz;
  const int wx = min(TW, n - x0), wy = min(P.ty, n - y0), zc = min(P.tz, n - z0);
  const int zend = z0 + zc;

  const int tid = threadIdx.x;
  const int ty = tid / P.tx;  // lanes past TX*TY (ty = TY) are idle
  const int tx = tid - ty * P.tx;
  const bool active = (tx * VX < wx) && (ty < wy);
  const int LX = TW + 2;
  const int plane = LX * (P.ty + 2);
  const int own = (min(ty, P.ty - 1) + 1) * LX + 1 + tx * VX;
  const size_t col = active ? size_t(y0 + ty) * n + (x0 + tx * VX) : size_t(y0) * n + x0;

  // halo job: 1 = VX-wide row segment above/below, 2 = the cell at element
  // VX - 1 of the aligned group left of the tile, 3 = element 0 of the
  // group right of it (columns and corners); 0 = none (own column re-read)
  int hjob = 0, hl = 0;
  size_t hcol = col;
  {
    const int TX = P.tx, TY = P.ty;
    int hx = -1, hy = 0;
    const int gl = (x0 - VX + n) % n, gr = (x0 + wx) % n;  // aligned groups
    const int yb = (y0 - 1 + n) % n, ya = (y0 + wy) % n;
    if (tid < TX) {
      if (tid * VX < wx) { hjob = 1; hx = x0 + tid * VX; hy = yb; hl = 1 + tid * VX; }
    } else if (tid < 2 * TX) {
      const int t = tid - TX;
      if (t * VX < wx) { hjob = 1; hx = x0 + t * VX; hy = ya; hl = (wy + 1) * LX + 1 + t * VX; }
    } else if (tid < 2 * TX + TY) {
      const int r = tid - 2 * TX;
      if (r < wy) { hjob = 2; hx = gl; hy = y0 + r; hl = (r + 1) * LX; }
    } else if (tid < 2 * TX + 2 * TY) {
      const int r = tid - 2 * TX - TY;
      if (r < wy) { hjob = 3; hx = gr; hy = y0 + r; hl = (r + 1) * LX + wx + 1; }
    } else if (tid < 2 * TX + 2 * TY + 4) {
      const int k = tid - 2 * TX - 2 * TY;
      hjob = (k & 1) ? 3 : 2;
      hx = (k & 1) ? gr : gl;
      hy = (k & 2) ? ya : yb;
      hl = ((k & 2) ? (wy + 1) * LX : 0) + ((k & 1) ? wx + 1 : 0);
    }
    if (hx >= 0) hcol = size_t(hy) * n + hx;
  }
  auto wrapz = [n](int z) { return z < 0 ? z + n : (z >= n ? z - n : z); };

  KSum acc_dd{0.0, 0.0}, acc_v{0.0, 0.0}, acc_p{0.0, 0.0};
  // ring: (f, F, C) of planes p-2 (A) and p-1 (B); momenta of plane p-1
  T fA[NF][VX], FA[NF][VX], CA[NF][VX], fB[NF][VX], FB[NF][VX], CB[NF][VX], qB[NF][VX];
  // raw loads in flight (plane p): own sites and halo group
  T nph[NF][VX], npi[NF][VX], hph[NF][VX], hpi[NF][VX];
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int v = 0; v < VX; ++v)
      fA[i][v] = FA[i][v] = CA[i][v] = fB[i][v] = FB[i][v] = CB[i][v] = qB[i][v] = T(0);

  auto load_plane = [&](int zz) {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const size_t o = (size_t(zz) * P.zs + i) * n2;
      const Vec<T, VX> u = ldv<T, VX>(phi_in + o + col), w = ldv<T, VX>(pi_in + o + col);
      const Vec<T, VX> hu = ldv<T, VX>(phi_in + o + hcol), hw = ldv<T, VX>(pi_in + o + hcol);
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        nph[i][v] = u.v[v];
        npi[i][v] = w.v[v];
        hph[i][v] = hu.v[v];
        hpi[i][v] = hw.v[v];
      }
    }
  };

  T* sink = static_cast<T*>(P.sink) + size_t(tid) * (2 * NF * VX);
  load_plane(wrapz(z0 - 1));
  // the stage scalars are formed while the first plane is in flight
  stage_scalars<CH>(P, C, tile_id, S, red_scratch, fresh, cp);
  c = static_cast<T>(S.c_next);
  alpha = static_cast<T>(S.alpha);
  beta = static_cast<T>(S.beta);
  if constexpr (kSplit) split_offsets<KIND, NF, T>(P, S, P.offs[C.p_out], tile_id, fbar, pibar, fbT, sk);
  // same trailing sequence as an iteration (loads, then 2 NF stores) so the
  // wait at the loop head covers the loads only
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    stv<T, VX>(sink + (2 * i) * VX, fB[i]);
    stv<T, VX>(sink + (2 * i + 1) * VX, qB[i]);
  }

  int buf = 0;
  for (int p = z0 - 1; p <= zend; ++p) {
    T* L = lds + size_t(buf) * NF * plane;
    T qN[NF][VX];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        qN[i][v] = npi[i][v];
        const T f = drift(nph[i][v], npi[i][v], c);
        if (active) L[i * plane + own + v] = f;
      }
      if (hjob == 1) {
#pragma unroll
        for (int v = 0; v < VX; ++v) L[i * plane + hl + v] = drift(hph[i][v], hpi[i][v], c);
      } else if (hjob >= 2) {
        const T f = hjob == 2 ? hph[i][VX - 1] : hph[i][0];
        const T q = hjob == 2 ? hpi[i][VX - 1] : hpi[i][0];
        L[i * plane + hl] = drift(f, q, c);
      }
    }
    __syncthreads();
    load_plane(wrapz(min(p + 1, zend)));  // past the end: the last plane again
    T fN[NF][VX], FN[NF][VX], CN[NF][VX];
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        const T* Li = L + i * plane + own + v;
        fN[i][v] = Li[0];
        FN[i][v] = (Li[-1] + Li[1]) + (Li[-LX] + Li[LX]);
        CN[i][v] = (Li[-LX - 1] + Li[-LX + 1]) + (Li[LX - 1] + Li[LX + 1]);
      }
    // sites at plane z = p - 1: ring (A, B, N) = planes (z - 1, z, z + 1)
    const bool out = active && p >= z0 + 1;
    {
      double dd = 0.0, p2 = 0.0, vs = 0.0;
      T pn[NF][VX];
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        T f[NF], D[NF], dV[NF], V;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          const T faces = FB[i][v] + (fA[i][v] + fN[i][v]);
          const T edges = CB[i][v] + (FA[i][v] + FN[i][v]);
          const T corners = CA[i][v] + CN[i][v];
          f[i] = fB[i][v];
          D[i] = ((w0 * f[i] + w1 * faces) + w2 * edges) + w3 * corners;
        }
        if constexpr (kSplit)
          potential_split<KIND, NF, T>(fbT, f, pot, sk, V, dV);
        else
          potential<KIND, NF, T>(f, pot, V, dV);
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          pn[i][v] = qB[i][v] + alpha * D[i] - beta * dV[i];
          if constexpr (kSplit) {
            dd += (fbar[i] + double(f[i])) * double(D[i]);
            const double q = pibar[i] + double(pn[i][v]);
            p2 += q * q;
          } else {
            dd += double(f[i]) * double(D[i]);
            p2 += double(pn[i][v]) * double(pn[i][v]);
          }
        }
        vs += double(V);
      }
      const size_t zo = size_t(wrapz(p - 1));
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const size_t oc = (zo * P.zs + i) * n2 + col;
        T* po = out ? phi_out + oc : sink + (2 * i) * VX;
        T* qo = out ? pi_out + oc : sink + (2 * i + 1) * VX;
        stv_mode<NT, T, VX>(po, fB[i]);
        stv_mode<NT, T, VX>(qo, pn[i]);
      }
      if (out) {
        kadd(acc_dd, dd);
        kadd(acc_v, vs);
        kadd(acc_p, p2);
      }
    }
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int v = 0; v < VX; ++v) {
        fA[i][v] = fB[i][v]; FA[i][v] = FB[i][v]; CA[i][v] = CB[i][v];
        fB[i][v] = fN[i][v]; FB[i][v] = FN[i][v]; CB[i][v] = CN[i][v];
        qB[i][v] = qN[i][v];
      }
    buf ^= 1;
  }

  KSum v3[3] = {acc_dd, acc_v, acc_p};
  block_reduce<3>(v3, red_scratch);
  if (threadIdx.x == 0) {
    double* o = P.partials[C.p_out] + size_t(tile_id) * 6;
    o[0] = v3[0].s; o[1] = v3[0].c;
    o[2] = v3[1].s; o[3] = v3[1].c;
    o[4] = v3[2].s; o[5] = v3[2].c;
  }
}

// ST: 0 = 7-point pass, 1 = any member of the cubic family (27-point pass),
// 2 = 7-point pass with non-temporal result stores, 3 = 27-point pass with
// non-temporal result stores.
// CH: the kernel can run chained (the solo pass; batches never chain).
template <typename T, int NF, int KIND, int VX, int PF, int ST, bool CH>
__device__ __forceinline__ void pass_any(const PassParams& P, const Chain& C, int tile_id, T* lds,
                                         KSum* red, DevScalars& S, bool fresh) {
  if constexpr (ST == 1 || ST == 3)
    pass_tile27<T, NF, KIND, VX, ST == 3, CH>(P, C, tile_id, lds, red, S, fresh);
  else
    pass_tile<T, NF, KIND, VX, PF, ST == 2, CH>(P, C, tile_id, lds, red, S, fresh);
}

template <typename T, int NF, int KIND, int VX, int PF, int ST>
__global__ __launch_bounds__(kBlock) void pass_kernel(PassParams P, Chain C) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ KSum red_scratch[4 * 3];
  __shared__ DevScalars S;
  pass_any<T, NF, KIND, VX, PF, ST, true>(P, C, xcd_tile(blockIdx.x, gridDim.x),
                                    reinterpret_cast<T*>(smem_raw), red_scratch, S, true);
}

// Batched form: the tiles of many lattices (same precision, potential family
// and per-lane shape; any sizes) in one launch.  Global tile g belongs to run
// r with start[r] <= g < start[r+1].  Each XCD takes a contiguous range of
// global tiles and its workgroups stride through it: with one workgroup per
// tile (the default launch) a workgroup takes one tile, at most two when
// the ranges are uneven; with a smaller, persistent grid each workgroup
// works through many.  A run's tiles and partial sums are exactly those of
// the same lattice advanced alone, whatever the grid.
template <typename T, int NF, int KIND, int VX, int PF, int ST>
__global__ __launch_bounds__(kBlock) void batched_pass_kernel(const PassParams* __restrict__ runs,
                                                             const int* __restrict__ start,
                                                             int nruns, Chain C) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ KSum red_scratch[4 * 3];
  __shared__ DevScalars S;
  // workgroups are dealt to the 8 XCDs round-robin; a grid of fewer than 8
  // spreads the tile list over the XCDs it has
  constexpr int kXcd = 8;
  const int total = start[nruns];
  const int G = gridDim.x, b = blockIdx.x;
  const int nx = G < kXcd ? G : kXcd;
  const int xcd = b % nx, i = b / nx;
  const int nbx = (G - xcd + nx - 1) / nx;  // workgroups on this XCD
  const int t0 = int((long long)total * xcd / nx);
  const int t1 = int((long long)total * (xcd + 1) / nx);
  int prev = -1;  // run of the previous tile: its stage scalars are still in S
  for (int g = t0 + i; g < t1; g += nbx) {
    int lo = 0, hi = nruns - 1;  // run with start[r] <= g < start[r + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    pass_any<T, NF, KIND, VX, PF, ST, false>(runs[lo], C, g - start[lo],
                                             reinterpret_cast<T*>(smem_raw),
                                      red_scratch, S, lo != prev);
    prev = lo;
  }
}

// ---------------------------------------------------------------------------
// Scalar updates.  They are written once and shared by the finalize and the
// begin kernel so that the operation sequence (hence every rounding) is the
// same whether a stage boundary falls inside one evolve call or between two.
// ---------------------------------------------------------------------------

// End of stage j: H3(w h) kick of p_a, H2(w h/2) kick of p_a, owed drift
// c = (w h/2)/a^2 of that H2, then H1(w h/2).
__device__ void end_stage(DevScalars& S, const BgConsts& K, const double* offs, double w,
                          double h, double SdD, double SV, double S2) {
#pragma clang fp contract(off)
  const double a = S.a_kick;
  const double tau = w * h;
  const double half = 0.5 * tau;
  if (K.split) {
    // the pass wrote the remainders around the offsets it recorded
    // (constant indices: S stays in registers, not in scratch memory)
#pragma unroll
    for (int i = 0; i < kMaxFields; ++i) {
      if (i < K.nf) {
        S.off_phi[i] = offs[i];
        S.off_pi[i] = offs[kMaxFields + i];
      }
    }
  }
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

// The scalar record is moved as 8-byte words, one per thread.
typedef double __attribute__((may_alias)) word_t;
constexpr int kScalarWords = int(sizeof(DevScalars) / sizeof(double));
static_assert(sizeof(DevScalars) % sizeof(double) == 0 && kScalarWords <= 64,
              "scalar record read as 8-byte words by the first wavefront");

// Second half of a stage update: publish this thread's scalar/offset word
// in LDS, reduce the partial sums over the workgroup, and let thread 0
// finish the stage.
__device__ void stage_update_finish(double word, KSum (&v)[3], const BgConsts& K, double w,
                                    double w_next, double h, int has_next, int end_of_step,
                                    bool record, KSum* scratch, DevScalars& S_io) {
  __shared__ double offs_sh[2 * kMaxFields];
  const int t = threadIdx.x;
  if (t < kScalarWords)
    reinterpret_cast<word_t*>(&S_io)[t] = word;
  else if (t >= 64 && t < 64 + 2 * kMaxFields)
    offs_sh[t - 64] = word;
  block_reduce<3>(v, scratch);  // its barriers publish the two LDS copies
  if (t == 0) {
    DevScalars S = S_io;
    const double SdD = v[0].s + v[0].c;
    const double SV = v[1].s + v[1].c;
    const double S2 = v[2].s + v[2].c;
    end_stage(S, K, offs_sh, w, h, SdD, SV, S2);
    S.parity ^= 1;
    if (end_of_step) S.eta = S.eta + h;
    if (end_of_step && S.hist != nullptr && S.hist_n < S.hist_cap) {
      // total density on this time slice from the first Friedmann equation
      // (2.18): rho = 3 m_pl^2 H^2 with H = a'/a^2 and a' = -p_a/(6 V_L m_pl^2)
      // (eq. (2.14))
      if (record) {
        const double hub = -S.p_a * K.inv6VLm2 / (S.a * S.a);
        double* r = S.hist + kHistRecord * S.hist_n;
        r[0] = S.eta;
        r[1] = S.a;
        r[2] = S.p_a;
        r[3] = 3.0 * K.mpl2 * hub * hub;
      }
      S.hist_n = S.hist_n + 1;
    }
    if (has_next) begin_stage(S, K, w_next, h);
    if (!(dev_finite(SdD) && dev_finite(SV) && dev_finite(S2) && dev_finite(S.a) &&
          dev_finite(S.p_a)))
      S.status |= kStatusNonFinite;
    S_io = S;
  }
}

// The word of the scalar record (threads 0 .. kScalarWords-1) or of the
// offset record (threads 64 .. 64 + 2 kMaxFields - 1) this thread publishes.
__device__ __forceinline__ double record_word(const DevScalars* sc, const double* offs) {
  const int t = threadIdx.x;
  if (t < kScalarWords) return reinterpret_cast<const word_t*>(sc)[t];
  if (t >= 64 && t < 64 + 2 * kMaxFields) return offs[t - 64];
  return 0.0;
}

// Finish stage (weight w) from the scalars *sc and the pass's partials
// and offset record, and begin the next (weight w_next) if has_next; eta
// += h when end_of_step.  The result is in S_io (LDS) once the caller's
// next barrier has passed; `record` writes the history record (the count
// advances either way).  The scalar record and the offset record are read
// by the workgroup together with the partials, so that the serial update
// of thread 0 waits on no memory.  Contains barriers: all threads call.
__device__ void stage_update(const DevScalars* sc, const double* partials, const double* offs,
                             int nblocks, const BgConsts& K, double w, double w_next, double h,
                             int has_next, int end_of_step, bool record, KSum* scratch,
                             DevScalars& S_io) {
  const double word = record_word(sc, offs);
  KSum v[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    const double* p = partials + size_t(b) * 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = kcombine(v[k], KSum{p[2 * k], p[2 * k + 1]});
  }
  stage_update_finish(word, v, K, w, w_next, h, has_next, end_of_step, record, scratch, S_io);
}

__device__ void finalize_body(const DevScalars* sc_in, DevScalars* sc_out, const double* partials,
                              const double* offs, int nblocks, const BgConsts& K, double w,
                              double w_next, double h, int has_next, int end_of_step,
                              KSum* scratch) {
  __shared__ DevScalars S;
  stage_update(sc_in, partials, offs, nblocks, K, w, w_next, h, has_next, end_of_step, true,
               scratch, S);
  if (threadIdx.x == 0) *sc_out = S;
}

static_assert(kChainMaxTiles <= 4 * kBlock, "ChainPre holds four tiles per thread");

__device__ void chain_prefetch(const PassParams& P, const Chain& C, ChainPre& cp) {
  const int t = threadIdx.x;
  cp.word = record_word(P.sc[C.s_in], P.offs[C.p_in]);
  const double* partials = P.partials[C.p_in];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int b = t + k * kBlock;
    if (b < P.ntiles) {
#pragma unroll
      for (int j = 0; j < 6; ++j) cp.p[k][j] = partials[size_t(b) * 6 + j];
    }
  }
}

template <bool CH>
__device__ void stage_scalars(const PassParams& P, const Chain& C, int tile_id, DevScalars& S,
                              KSum* scratch, bool fresh, const ChainPre& cp) {
  if (!fresh) return;  // S already holds this run's scalars (uniform branch)
  if (CH && C.chain) {
    // every workgroup finishes the previous stage the same way (the same
    // partials combined in the same order as stage_update); the first tile
    // keeps the result (and the history record) for the next launch
    KSum v[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (int(threadIdx.x) + k * kBlock < P.ntiles) {
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] = kcombine(v[q], KSum{cp.p[k][2 * q], cp.p[k][2 * q + 1]});
      }
    }
    stage_update_finish(cp.word, v, P.bg, C.w_prev, C.w, C.h, 1, C.eos, tile_id == 0, scratch, S);
    if (threadIdx.x == 0 && tile_id == 0) *P.sc[C.s_out] = S;
  } else if (threadIdx.x < kScalarWords) {
    reinterpret_cast<word_t*>(&S)[threadIdx.x] =
        reinterpret_cast<const word_t*>(P.sc[C.s_in])[threadIdx.x];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void stage_finalize_kernel(const DevScalars* sc_in,
                                                               DevScalars* sc_out,
                                                               const double* partials,
                                                               const double* offs, int nblocks,
                                                               BgConsts K, double w, double w_next,
                                                               double h, int has_next,
                                                               int end_of_step) {
  __shared__ KSum scratch[4 * 3];
  finalize_body(sc_in, sc_out, partials, offs, nblocks, K, w, w_next, h, has_next, end_of_step,
                scratch);
}

// One workgroup per run of a batch.
__global__ __launch_bounds__(kBlock) void batched_finalize_kernel(const BatchRun* __restrict__ runs,
                                                                 int s_in, int p_in, double w,
                                                                 double w_next, double h,
                                                                 int has_next, int end_of_step) {
  __shared__ KSum scratch[4 * 3];
  const BatchRun& R = runs[blockIdx.x];
  finalize_body(R.sc[s_in], R.sc[0], R.partials[p_in], R.offs[p_in], R.ntiles, R.bg, w, w_next, h,
                has_next, end_of_step, scratch);
}

__global__ void batched_begin_kernel(const BatchRun* __restrict__ runs, int nruns, double w,
                                     double h) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nruns) {
    DevScalars S = *runs[r].sc[0];
    begin_stage(S, runs[r].bg, w, h);
    *runs[r].sc[0] = S;
  }
}

__global__ void begin_kernel(DevScalars* sc, BgConsts K, double w, double h) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    DevScalars S = *sc;
    begin_stage(S, K, w, h);
    *sc = S;
  }
}

PassParams make_params(const LatView& v) {
  PassParams P;
  for (int k = 0; k < 2; ++k) {
    P.phi[k] = v.phi[k];
    P.pi[k] = v.pi[k];
    P.phi_w[k] = v.phi[k];
    P.pi_w[k] = v.pi[k];
  }
  P.sc[0] = v.sc;
  P.sc[1] = v.sc1;
  P.partials[0] = v.partials;
  P.partials[1] = v.partials1;
  P.offs[0] = v.offs;
  P.offs[1] = v.offs1;
  P.bg = v.bg;
  P.ntiles = v.tile.nblocks();
  P.sink = v.sink;
  P.prm = v.prm;
  for (int k = 0; k < 4; ++k) P.stc[k] = v.st.c[k];
  P.n = v.n;
  P.tx = v.tile.tx;
  P.ty = v.tile.ty;
  P.tz = v.tile.tz;
  P.ntx = v.tile.ntx;
  P.nty = v.tile.nty;
  P.ntz = v.tile.ntz;
  P.zs = v.zs;
  return P;
}

using PassFn = void (*)(PassParams, Chain);
using BatchedFn = void (*)(const PassParams*, const int*, int, Chain);

struct PassKernel {
  PassFn fn;
  BatchedFn bfn;
  size_t lds;
};

template <typename T, int NF, int KIND>
PassKernel pick_t(const Tile& t, int st) {
  PassKernel k;
  k.lds = size_t(2) * NF * (t.tx * t.vx + 2) * (t.ty + 2) * sizeof(T);
  if (st != 0) {
    // any cubic-family stencil: lagged (f, F, C) ring (see pass_tile27); two
    // sites per lane for up to two fields
    if constexpr (NF <= 2) {
      if (t.vx == 2) {
        k.fn = pf_nt(t.pf) ? pass_kernel<T, NF, KIND, 2, 1, 3> : pass_kernel<T, NF, KIND, 2, 1, 1>;
        k.bfn = pf_nt(t.pf) ? batched_pass_kernel<T, NF, KIND, 2, 1, 3>
                            : batched_pass_kernel<T, NF, KIND, 2, 1, 1>;
        return k;
      }
    }
    k.fn = pass_kernel<T, NF, KIND, 1, 1, 1>;
    k.bfn = batched_pass_kernel<T, NF, KIND, 1, 1, 1>;
    return k;
  }
  if constexpr (NF <= 2) {
    const int depth = pf_depth(t.pf);
    if (pf_nt(t.pf) && t.vx >= 2) {
      // non-temporal result stores (2 or 4 sites per lane)
      if (depth == 3) {
        k.fn = t.vx == 4 ? pass_kernel<T, NF, KIND, 4, 3, 2> : pass_kernel<T, NF, KIND, 2, 3, 2>;
        k.bfn = t.vx == 4 ? batched_pass_kernel<T, NF, KIND, 4, 3, 2>
                          : batched_pass_kernel<T, NF, KIND, 2, 3, 2>;
      } else if (depth == 2) {
        k.fn = t.vx == 4 ? pass_kernel<T, NF, KIND, 4, 2, 2> : pass_kernel<T, NF, KIND, 2, 2, 2>;
        k.bfn = t.vx == 4 ? batched_pass_kernel<T, NF, KIND, 4, 2, 2>
                          : batched_pass_kernel<T, NF, KIND, 2, 2, 2>;
      } else {
        k.fn = t.vx == 4 ? pass_kernel<T, NF, KIND, 4, 1, 2> : pass_kernel<T, NF, KIND, 2, 1, 2>;
        k.bfn = t.vx == 4 ? batched_pass_kernel<T, NF, KIND, 4, 1, 2>
                          : batched_pass_kernel<T, NF, KIND, 2, 1, 2>;
      }
    } else if (depth == 2) {
      k.fn = t.vx == 4 ? pass_kernel<T, NF, KIND, 4, 2, 0>
                       : (t.vx == 2 ? pass_kernel<T, NF, KIND, 2, 2, 0>
                                    : pass_kernel<T, NF, KIND, 1, 2, 0>);
      k.bfn = t.vx == 4 ? batched_pass_kernel<T, NF, KIND, 4, 2, 0>
                        : (t.vx == 2 ? batched_pass_kernel<T, NF, KIND, 2, 2, 0>
                                     : batched_pass_kernel<T, NF, KIND, 1, 2, 0>);
    } else {
      k.fn = t.vx == 4 ? pass_kernel<T, NF, KIND, 4, 1, 0>
                       : (t.vx == 2 ? pass_kernel<T, NF, KIND, 2, 1, 0>
                                    : pass_kernel<T, NF, KIND, 1, 1, 0>);
      k.bfn = t.vx == 4 ? batched_pass_kernel<T, NF, KIND, 4, 1, 0>
                        : (t.vx == 2 ? batched_pass_kernel<T, NF, KIND, 2, 1, 0>
                                     : batched_pass_kernel<T, NF, KIND, 1, 1, 0>);
    }
  } else {
    // more than two fields: one site per lane, no deep prefetch (register budget)
    k.fn = pass_kernel<T, NF, KIND, 1, 1, 0>;
    k.bfn = batched_pass_kernel<T, NF, KIND, 1, 1, 0>;
  }
  return k;
}

template <typename T>
PassKernel pick_prec(int pot, int nf, const Tile& t, int st) {
  switch (pot) {
    case SL_POT_CHAOTIC2: return pick_t<T, 2, SL_POT_CHAOTIC2>(t, st);
    case SL_POT_OSCILLON: return pick_t<T, 1, SL_POT_OSCILLON>(t, st);
    case SL_POT_QBALL_LOG: return pick_t<T, 2, SL_POT_QBALL_LOG>(t, st);
    default: break;
  }
  switch (nf) {
    case 1: return pick_t<T, 1, SL_POT_FREE>(t, st);
    case 2: return pick_t<T, 2, SL_POT_FREE>(t, st);
    case 3: return pick_t<T, 3, SL_POT_FREE>(t, st);
    case 4: return pick_t<T, 4, SL_POT_FREE>(t, st);
    case 5: return pick_t<T, 5, SL_POT_FREE>(t, st);
    case 6: return pick_t<T, 6, SL_POT_FREE>(t, st);
    case 7: return pick_t<T, 7, SL_POT_FREE>(t, st);
    default: return pick_t<T, 8, SL_POT_FREE>(t, st);
  }
}

PassKernel pick(int prec, int pot, int nf, const Tile& t, int st) {
  return prec == SL_FP32 ? pick_prec<float>(pot, nf, t, st) : pick_prec<double>(pot, nf, t, st);
}

}  // namespace

hipError_t launch_pass(const LatView& v, const Chain& c, hipStream_t s) {
  if (v.nf < 1 || v.nf > kMaxFields) return hipErrorInvalidValue;
  if (!pf_valid(v.tile.pf)) return hipErrorInvalidValue;
  if (v.nf > 2 && (v.tile.vx != 1 || v.tile.pf != 1)) return hipErrorInvalidValue;
  if (v.st.kind != 0 && (v.tile.vx > 2 || (v.tile.pf != 1 && v.tile.pf != (1 | kPfNontemporal))))
    return hipErrorInvalidValue;
  if (pf_nt(v.tile.pf) && v.tile.vx < 2) return hipErrorInvalidValue;
  // the 27-point pass needs lanes for 2 rows + 2 columns + 4 corners of halo
  if (v.st.kind != 0 && 2 * v.tile.tx + 2 * v.tile.ty + 4 > kBlock) return hipErrorInvalidValue;
  if (c.chain && v.tile.nblocks() > kChainMaxTiles) return hipErrorInvalidValue;
  const PassKernel k = pick(v.prec, v.pot, v.nf, v.tile, v.st.kind);
  hipLaunchKernelGGL(k.fn, dim3(v.tile.nblocks()), dim3(kBlock), k.lds, s, make_params(v), c);
  return hipGetLastError();
}

PassParams pass_params(const LatView& v) { return make_params(v); }

hipError_t launch_batched_pass(int prec, int pot, int nf, const Tile& shape, int stencil_kind,
                               size_t lds, const PassParams* runs_dev, const int* start_dev,
                               int nruns, int grid, const Chain& c, hipStream_t s) {
  const PassKernel k = pick(prec, pot, nf, shape, stencil_kind);
  hipLaunchKernelGGL(k.bfn, dim3(grid), dim3(kBlock), lds, s, runs_dev, start_dev, nruns, c);
  return hipGetLastError();
}

int batched_blocks_per_cu(int prec, int pot, int nf, const Tile& shape, int stencil_kind,
                          size_t lds) {
  const PassKernel k = pick(prec, pot, nf, shape, stencil_kind);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k.bfn, kBlock, lds) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

size_t pass_lds_bytes(int prec, int nf, const Tile& t) {
  return size_t(2) * nf * (t.tx * t.vx + 2) * (t.ty + 2) * (prec == SL_FP32 ? 4 : 8);
}

hipError_t launch_batched_finalize(const BatchRun* runs_dev, int nruns, int s_in, int p_in,
                                   double w, double w_next, double h, int has_next,
                                   int end_of_step, hipStream_t s) {
  hipLaunchKernelGGL(batched_finalize_kernel, dim3(nruns), dim3(kBlock), 0, s, runs_dev, s_in, p_in,
                     w, w_next, h, has_next, end_of_step);
  return hipGetLastError();
}

hipError_t launch_batched_begin(const BatchRun* runs_dev, int nruns, double w, double h,
                                hipStream_t s) {
  hipLaunchKernelGGL(batched_begin_kernel, dim3((nruns + 255) / 256), dim3(256), 0, s, runs_dev,
                     nruns, w, h);
  return hipGetLastError();
}

int pass_blocks_per_cu(int prec, int pot, int nf, const Tile& t, int stencil_kind) {
  const PassKernel k = pick(prec, pot, nf, t, stencil_kind);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k.fn, kBlock, k.lds) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

hipError_t launch_stage_finalize(const LatView& v, int s_in, int p_in, double w, double w_next,
                                 double h, int has_next, int end_of_step, hipStream_t s) {
  hipLaunchKernelGGL(stage_finalize_kernel, dim3(1), dim3(kBlock), 0, s, s_in ? v.sc1 : v.sc, v.sc,
                     p_in ? v.partials1 : v.partials, p_in ? v.offs1 : v.offs, v.tile.nblocks(),
                     v.bg, w, w_next, h, has_next, end_of_step);
  return hipGetLastError();
}

hipError_t launch_begin(const LatView& v, double w, double h, hipStream_t s) {
  hipLaunchKernelGGL(begin_kernel, dim3(1), dim3(64), 0, s, v.sc, v.bg, w, h);
  return hipGetLastError();
}

}  // namespace symlat
