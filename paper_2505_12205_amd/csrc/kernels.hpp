// kernels.hpp -- gfx950 device code of the phase-field LBM step.
//
// One step at parity P (P = steps % 2) is, over a table of domains,
//   kb_interior<P, PHI>, kb_faces<P, PHI>: phi(x) = sum_a h_a(x) (Eq. phase_field_variable)
//   kb_interior<P, STEP>, kb_faces<P, STEP>: stencil of phi, macroscopic update,
//       both collisions and the in-place AA streaming of both population sets;
//       the hydrodynamic set relaxes with WMRT, or with BGK (template flag)
//   kb_outlet<P>: convective outflow plane (only with an outlet face)
// Nodes off the y and z faces of non-periodic axes take the fast path with
// precomputed neighbour offsets (x walls included, with a per-lane slot
// choice): in D3Q19 the kernel marches each tile along z with the tile's
// phase field and its halo staged in an LDS ring of planes (kb_march), in
// D2Q9 (and with marching switched off) one tile per block reads the stencil
// from global memory (kb_interior); the y and z face layers take the general
// path.
//
// Storage is structure-of-arrays, pop[a][node] with node = x + nx*(y + ny*z)
// (x fastest), one array per set; streaming is the AA pattern:
//   even step: read  pop[a][x],           write pop[abar][x]
//   odd step : read  pop[abar][x - e_a],  write pop[a][x + e_a]
// so every step reads and writes each population slot once, in place.  At
// halfway walls the slot that the missing neighbour would have used is used
// instead (bounce-back: pop[a][x]; specular reflection: the reflected slot of
// the tangential neighbour), which keeps the read and write sets of each node
// identical and the update race-free.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbm {

enum { BC_PERIODIC = 0, BC_NOSLIP = 1, BC_FREESLIP = 2, BC_INLET = 3, BC_OUTLET = 4 };

struct KParams {
  int nx, ny, nz, N;       // grid, nodes
  int plane;               // nodes of an inlet/outlet plane
  float rho_l, drho;       // rho = rho_l + phi drho
  float tau_l, dtau;       // tau = tau_l + phi dtau
  float beta4, kappa;      // 4 beta, kappa of the chemical potential
  float inv_xi, omega_h;   // 1/xi, 1/(tau_phi + 1/2)
  float gx, gy, gz, fb_rhol;  // F_b = (rho - fb_rhol) g
  int bc[6];
  float in_c0, in_c1, in_R, in_u, two_over_xi;
  int clamp;
  int has_inlet, has_outlet;
  int outlet_mode;         // convective velocity: 0 local, 1 plane maximum, 2 plane average
  int wbits, nsbits;       // x faces: bit 0 (1) = the minus (plus) face is a wall / a no-slip wall
};

struct KBufs {
  void* h;                 // Q*N populations (storage type of the codec)
  void* g;
  float* u;                // 3*N, u[d*N + node]
  const float* phi;        // phase field of this step (stencil)
  float* phi_out;          // written by k_phi
  const float* ref;        // 16-bit forms: phase field (previous step) of each stored value's reader
  float* obuf;             // outlet plane: h then g, (2Q) * plane
};

// ---------------------------------------------------------------------------
// population codecs
// ---------------------------------------------------------------------------
template <int ST>
struct Codec;

// The interior kernels address the populations, phase field and velocity
// through global-address-space pointers: the buffers come from a device-side
// domain table, and without the qualifier every access would be a generic
// (flat) one.  The codecs take either pointer kind.

// store with an optional non-temporal hint (the written populations are not
// read again within the step, so they need not stay in L2)
template <bool NT, typename P, typename I, typename T>
__device__ __forceinline__ void put(P p, I i, T v) {
  if (NT)
    __builtin_nontemporal_store(v, p + i);
  else
    p[i] = v;
}

template <>
struct Codec<0> {  // FP32 as is
  using T = float;
  template <typename P, typename I>
  static __device__ __forceinline__ float ld_h(P p, I i, float w, float ref) { return p[i]; }
  template <bool NT = false, typename P = void, typename I = size_t>
  static __device__ __forceinline__ void st_h(P p, I i, float v, float iw, float ref) { put<NT>(p, i, (T)v); }
  template <typename P, typename I>
  static __device__ __forceinline__ float ld_g(P p, I i, float w) { return p[i]; }
  template <bool NT = false, typename P = void, typename I = size_t>
  static __device__ __forceinline__ void st_g(P p, I i, float v, float iw) { put<NT>(p, i, (T)v); }
};

template <>
struct Codec<1> {  // FP16 deviations: h -> h/w - phi_ref, g -> g/w
  using T = _Float16;
  template <typename P, typename I>
  static __device__ __forceinline__ float ld_h(P p, I i, float w, float ref) {
    return w * ((float)p[i] + ref);
  }
  template <bool NT = false, typename P = void, typename I = size_t>
  static __device__ __forceinline__ void st_h(P p, I i, float v, float iw, float ref) {
    put<NT>(p, i, (T)(v * iw - ref));
  }
  template <typename P, typename I>
  static __device__ __forceinline__ float ld_g(P p, I i, float w) { return w * (float)p[i]; }
  template <bool NT = false, typename P = void, typename I = size_t>
  static __device__ __forceinline__ void st_g(P p, I i, float v, float iw) { put<NT>(p, i, (T)(v * iw)); }
};

__device__ __forceinline__ uint16_t f2bf(float v) {  // round to nearest even
  uint32_t b = __float_as_uint(v);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// BF16 with stochastic rounding: 16 pseudo-random bits, a hash of the value's
// FP32 bits and its slot index, are added below the kept significand before
// truncation, so the stored value rounds up with probability equal to the
// dropped fraction (unbiased on average; deterministic for given inputs, and
// the slot index is local to the domain, so a batched domain stores the same
// bits as the domain alone).  Round-to-nearest-even biases the hydrodynamic
// set's small velocity moments step after step; this removes the bias.
// One 32-bit multiply: the carries make the product's upper half a
// nonlinear mix of every input bit (a shift-xor mix alone left the rounding
// correlated with the dropped bits and biased).
__device__ __forceinline__ uint16_t f2bf_sr(float v, uint32_t slot) {
  const uint32_t b = __float_as_uint(v);
  const uint32_t x = (b + (slot << 16) + slot) * 0x85EBCA77u;
  return (uint16_t)((b + (x >> 16)) >> 16);
}

template <>
struct Codec<2> {  // BF16 deviations, same encoding as FP16, stochastic rounding
  using T = uint16_t;
  template <typename P, typename I>
  static __device__ __forceinline__ float ld_h(P p, I i, float w, float ref) {
    return w * (bf2f(p[i]) + ref);
  }
  template <bool NT = false, typename P = void, typename I = size_t>
  static __device__ __forceinline__ void st_h(P p, I i, float v, float iw, float ref) {
    put<NT>(p, i, f2bf_sr(v * iw - ref, (uint32_t)i));
  }
  template <typename P, typename I>
  static __device__ __forceinline__ float ld_g(P p, I i, float w) { return w * bf2f(p[i]); }
  template <bool NT = false, typename P = void, typename I = size_t>
  static __device__ __forceinline__ void st_g(P p, I i, float v, float iw) {
    put<NT>(p, i, f2bf_sr(v * iw, (uint32_t)i));
  }
};

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int node_of(const KParams& P, int x, int y, int z) {
  return x + P.nx * (y + P.ny * z);
}
__device__ __forceinline__ int dim_of(const KParams& P, int d) { return d == 0 ? P.nx : (d == 1 ? P.ny : P.nz); }

// Source of population a entering node c: the slot it is read from and the
// node that produced it (for the 16-bit decode).  Returns false if the source
// lies beyond the inlet or outlet face (the value then comes from that
// boundary condition).
template <int Q, int ODD>
__device__ __forceinline__ bool resolve_src(const KParams& P, const int c[3], int a, int& slot_pop,
                                            int& slot_node, int& src_node) {
  int s[3];
  int mask = 0;
  bool noslip = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e = ecomp<Q>(a, d);
    s[d] = c[d] - e;
    if (e == 0) continue;
    const int n = dim_of(P, d);
    if (s[d] < 0 || s[d] >= n) {
      const int b = P.bc[2 * d + (s[d] >= n ? 1 : 0)];
      if (b == BC_PERIODIC) {
        s[d] = s[d] < 0 ? s[d] + n : s[d] - n;
      } else if (b == BC_INLET || b == BC_OUTLET) {
        return false;
      } else {
        mask |= 1 << d;
        noslip |= (b == BC_NOSLIP);
      }
    }
  }
  if (mask == 0) {
    src_node = node_of(P, s[0], s[1], s[2]);
    slot_pop = ODD ? Lat<Q>::opp[a] : a;
    slot_node = ODD ? src_node : node_of(P, c[0], c[1], c[2]);
    return true;
  }
  const int self = node_of(P, c[0], c[1], c[2]);
  if (noslip) {  // halfway bounce-back: post-collision abar of this node
    src_node = self;
    slot_pop = a;
    slot_node = self;
    return true;
  }
  // halfway specular reflection: post-collision reflect(a) of x - e_{a,t}
  int t[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) t[d] = (mask >> d & 1) ? c[d] : s[d];
  src_node = node_of(P, t[0], t[1], t[2]);
  int r = a;
  switch (mask) {  // constant-folded per a
    case 1: r = reflect<Q>(a, 1); break;
    case 2: r = reflect<Q>(a, 2); break;
    case 3: r = reflect<Q>(a, 3); break;
    case 4: r = reflect<Q>(a, 4); break;
    case 5: r = reflect<Q>(a, 5); break;
    case 6: r = reflect<Q>(a, 6); break;
    default: r = reflect<Q>(a, 7); break;
  }
  slot_pop = ODD ? Lat<Q>::opp[r] : a;
  slot_node = ODD ? src_node : self;
  return true;
}

// Destination slot of post-collision population a leaving node c; false if it
// leaves through the inlet or outlet face.
template <int Q, int ODD>
__device__ __forceinline__ bool resolve_dst(const KParams& P, const int c[3], int a, int& slot_pop,
                                            int& slot_node) {
  if (!ODD) {
    slot_pop = Lat<Q>::opp[a];
    slot_node = node_of(P, c[0], c[1], c[2]);
    return true;
  }
  int t[3];
  int mask = 0;
  bool noslip = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e = ecomp<Q>(a, d);
    t[d] = c[d] + e;
    if (e == 0) continue;
    const int n = dim_of(P, d);
    if (t[d] < 0 || t[d] >= n) {
      const int b = P.bc[2 * d + (t[d] >= n ? 1 : 0)];
      if (b == BC_PERIODIC) {
        t[d] = t[d] < 0 ? t[d] + n : t[d] - n;
      } else if (b == BC_INLET || b == BC_OUTLET) {
        return false;
      } else {
        mask |= 1 << d;
        noslip |= (b == BC_NOSLIP);
      }
    }
  }
  if (mask == 0) {
    slot_pop = a;
    slot_node = node_of(P, t[0], t[1], t[2]);
    return true;
  }
  if (noslip) {
    slot_pop = Lat<Q>::opp[a];
    slot_node = node_of(P, c[0], c[1], c[2]);
    return true;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (mask >> d & 1) t[d] = c[d];
  int r = a;
  switch (mask) {
    case 1: r = reflect<Q>(a, 1); break;
    case 2: r = reflect<Q>(a, 2); break;
    case 3: r = reflect<Q>(a, 3); break;
    case 4: r = reflect<Q>(a, 4); break;
    case 5: r = reflect<Q>(a, 5); break;
    case 6: r = reflect<Q>(a, 6); break;
    default: r = reflect<Q>(a, 7); break;
  }
  slot_pop = r;
  slot_node = node_of(P, t[0], t[1], t[2]);
  return true;
}

// Node that receives post-collision population a of node c after streaming
// (the reader of the stored value at the next step).  Returns 0 if it leaves
// the domain through the inlet or outlet, 1 for the plain (possibly
// periodically wrapped) neighbour c + e_a, 2 for a wall-reflected target.
template <int Q>
__device__ __forceinline__ int stream_target(const KParams& P, const int c[3], int a, int& node) {
  int t[3];
  int mask = 0;
  bool noslip = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e = ecomp<Q>(a, d);
    t[d] = c[d] + e;
    if (e == 0) continue;
    const int n = dim_of(P, d);
    if (t[d] < 0 || t[d] >= n) {
      const int b = P.bc[2 * d + (t[d] >= n ? 1 : 0)];
      if (b == BC_PERIODIC) {
        t[d] = t[d] < 0 ? t[d] + n : t[d] - n;
      } else if (b == BC_INLET || b == BC_OUTLET) {
        return 0;
      } else {
        mask |= 1 << d;
        noslip |= (b == BC_NOSLIP);
      }
    }
  }
  if (mask == 0) {
    node = node_of(P, t[0], t[1], t[2]);
    return 1;
  }
  if (noslip) {
    node = node_of(P, c[0], c[1], c[2]);
    return 2;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (mask >> d & 1) t[d] = c[d];
  node = node_of(P, t[0], t[1], t[2]);
  return 2;
}

// nozzle profile psi = 1/2 [1 + tanh(2 (R - r)/xi)] at tangential position (p0, p1)
__device__ __forceinline__ float inlet_psi(const KParams& P, float p0, float p1) {
  const float d0 = p0 - P.in_c0, d1 = p1 - P.in_c1;
  const float r = sqrtf(d0 * d0 + d1 * d1);
  return 0.5f * (1.0f + tanhf(P.two_over_xi * (P.in_R - r)));
}

// tangential coordinates of node c on the inlet face
template <int Q>
__device__ __forceinline__ void inlet_tangential(const int c[3], float& p0, float& p1) {
  if (Lat<Q>::D == 3) {
    p0 = (float)c[0];
    p1 = (float)c[1];
  } else {
    p0 = (float)c[0];
    p1 = 0.0f;
  }
}

// phi at c + e_a with the ghost rules: periodic wrap; walls and outlet take
// the adjacent fluid value; the inlet takes phi_in.
template <int Q>
__device__ __forceinline__ float phi_nb(const KParams& P, const float* __restrict__ phi, const int c[3],
                                        int a) {
  int t[3];
  bool inlet = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e = ecomp<Q>(a, d);
    t[d] = c[d] + e;
    if (e == 0) continue;
    const int n = dim_of(P, d);
    if (t[d] < 0 || t[d] >= n) {
      const int b = P.bc[2 * d + (t[d] >= n ? 1 : 0)];
      if (b == BC_PERIODIC) {
        t[d] = t[d] < 0 ? t[d] + n : t[d] - n;
      } else {
        t[d] = t[d] < 0 ? 0 : n - 1;
        inlet |= (b == BC_INLET);
      }
    }
  }
  if (inlet) {
    float p0, p1;
    inlet_tangential<Q>(t, p0, p1);
    return inlet_psi(P, p0, p1);
  }
  return phi[node_of(P, t[0], t[1], t[2])];
}

template <int Q>
__device__ __forceinline__ bool is_inlet_node(const KParams& P, const int c[3]) {
  return P.has_inlet && c[Lat<Q>::AX] == 0;
}
template <int Q>
__device__ __forceinline__ bool is_outlet_node(const KParams& P, const int c[3]) {
  return P.has_outlet && c[Lat<Q>::AX] == dim_of(P, Lat<Q>::AX) - 1;
}
template <int Q>
__device__ __forceinline__ int plane_index(const KParams& P, const int c[3]) {
  return Lat<Q>::D == 3 ? c[0] + P.nx * c[1] : c[0];
}

// Velocity inlet (appendix B) at node c: fills the unknown populations
// (e_a along the inward normal > 0) from the known ones, for both sets.
template <int Q>
__device__ __forceinline__ void apply_inlet(const KParams& P, const int c[3], float* h, float* g) {
  constexpr int AX = Lat<Q>::AX;
  float p0, p1;
  inlet_tangential<Q>(c, p0, p1);
  const float psi = inlet_psi(P, p0, p1);
  const float un = P.in_u * psi;  // u_in along +AX
  const float rho_in = P.rho_l + psi * P.drho;
  const float fb = (rho_in - P.fb_rhol);
  const float F[3] = {fb * P.gx, fb * P.gy, fb * P.gz};
  const float inv_rho3 = 3.0f / rho_in;
  float feq[Q], heq[Q], Fa[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const float eu = ecomp<Q>(a, AX) * un;
    const float w = Lat<Q>::w[a];
    feq[a] = w * (3.0f * eu + 4.5f * eu * eu - 1.5f * un * un);
    heq[a] = psi * w * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * un * un);
    Fa[a] = w * inv_rho3 * (ecomp<Q>(a, 0) * F[0] + ecomp<Q>(a, 1) * F[1] + ecomp<Q>(a, 2) * F[2]);
  }
  float M[3] = {0.f, 0.f, 0.f};
  float theta = 0.f;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    if (ecomp<Q>(a, AX) != 0) continue;
    const float fp = g[a] + 0.5f * Fa[a] - feq[a];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (ecomp<Q>(a, d) != 0) M[d] += ecomp<Q>(a, d) * fp;
    theta += h[a] - heq[a];
  }
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    if (ecomp<Q>(a, AX) <= 0) continue;
    const int b = Lat<Q>::opp[a];
    const float eM = ecomp<Q>(a, 0) * M[0] + ecomp<Q>(a, 1) * M[1] + ecomp<Q>(a, 2) * M[2];
    const float fpa = (g[b] + 0.5f * Fa[b]) + (feq[a] - feq[b]) - 0.5f * eM;
    g[a] = fpa - 0.5f * Fa[a];
    bool tang = false;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d != AX && ecomp<Q>(a, d) != 0) tang = true;
    h[a] = heq[a] - (h[b] - heq[b]) - (tang ? theta * (1.0f / Lat<Q>::NH) : 0.0f);
  }
}

// Load the post-stream populations of node c for a step of parity ODD.
template <int Q, int ST, int ODD, bool LOAD_G>
__device__ __forceinline__ void load_node(const KParams& P, const KBufs& B, const int c[3], float* h,
                                          float* g) {
  using C = Codec<ST>;
  using T = typename C::T;
  const T* H = (const T*)B.h;  // not restrict: the same arrays are written in place
  const T* G = (const T*)B.g;
  const size_t N = (size_t)P.N;
  if (is_outlet_node<Q>(P, c)) {
    const int pi = plane_index<Q>(P, c);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      h[a] = B.obuf[(size_t)a * P.plane + pi];
      if (LOAD_G) g[a] = B.obuf[(size_t)(Q + a) * P.plane + pi];
    }
    return;
  }
  const bool inlet = is_inlet_node<Q>(P, c);
  // 16-bit forms: every stored h value was encoded relative to the phase
  // field (previous step) of the node that reads it, i.e. this node
  const float ref = (ST == 0) ? 0.0f : B.ref[node_of(P, c[0], c[1], c[2])];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int sp, sn, src;
    if (resolve_src<Q, ODD>(P, c, a, sp, sn, src)) {
      h[a] = C::ld_h(H, (size_t)sp * N + sn, Lat<Q>::w[a], ref);
      if (LOAD_G) g[a] = C::ld_g(G, (size_t)sp * N + sn, Lat<Q>::w[a]);
    } else {
      h[a] = 0.0f;
      if (LOAD_G) g[a] = 0.0f;
    }
  }
  if (inlet && LOAD_G) apply_inlet<Q>(P, c, h, g);
}

// XCD-aware tile order: consecutive hardware block ids go round-robin to the
// 8 XCDs; remap so that each XCD walks a contiguous range of tiles (and its
// L2 holds the phase-field planes its tiles share).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int per = nblocks / 8, rem = nblocks % 8;
  const int xcd = b % 8, k = b / 8;
  return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

struct Tiling {
  int bx, by, ntx, nty, ntiles;
};

__device__ __forceinline__ bool tile_coords(const KParams& P, const Tiling& T, int c[3]) {
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = L % T.ntx;
  const int r = L / T.ntx;
  const int ty = r % T.nty;
  c[2] = r / T.nty;
  c[0] = tx * T.bx + (int)threadIdx.x % T.bx;
  c[1] = ty * T.by + (int)threadIdx.x / T.bx;
  return c[0] < P.nx && c[1] < P.ny;
}

// Kahan-compensated sum v[0] + ... + v[Q-1] = hi + lo
template <int Q>
__device__ __forceinline__ void kahan_sum(const float* v, float& hi, float& lo) {
  float s = 0.0f, c = 0.0f;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const float y = v[a] - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  hi = s;
  lo = -c;
}

// ---------------------------------------------------------------------------
// node physics (shared by the fast interior path and the general path)
// ---------------------------------------------------------------------------
struct Stress {  // second moments sum g e e
  float xx, yy, zz, xy, yz, xz;
};

// Viscous force of the WMRT operator (Eq. viscous_force_wmrt) in the closed
// form -tau [s dev(Pi) + tr(Pi)/d I] grad rho, Pi = sum e e (g - f^eq(p*, u)):
// the weighted moment basis makes M^-1 S M act as s on the deviatoric
// second moments and as 1 on their trace.  BGK (Eq. viscous_force_bgk):
// -tau s Pi grad rho, the trace relaxed at s as well.
template <int D, bool BGK>
__device__ __forceinline__ void viscous_force(const Stress& S, float p, const float u[3], float tau,
                                              float s, const float gr[3], float F[3]) {
  const float p3 = p * (1.0f / 3.0f);
  const float xx = S.xx - p3 - u[0] * u[0];
  const float yy = S.yy - p3 - u[1] * u[1];
  const float zz = (D == 3) ? S.zz - p3 - u[2] * u[2] : 0.0f;
  const float xy = S.xy - u[0] * u[1];
  const float yz = (D == 3) ? S.yz - u[1] * u[2] : 0.0f;
  const float xz = (D == 3) ? S.xz - u[0] * u[2] : 0.0f;
  const float tr = BGK ? 0.0f : (xx + yy + zz) * (1.0f / D);
  const float Txx = s * (xx - tr) + tr, Tyy = s * (yy - tr) + tr, Tzz = s * (zz - tr) + tr;
  const float Txy = s * xy, Tyz = s * yz, Txz = s * xz;
  F[0] = -tau * (Txx * gr[0] + Txy * gr[1] + Txz * gr[2]);
  F[1] = -tau * (Txy * gr[0] + Tyy * gr[1] + Tyz * gr[2]);
  F[2] = (D == 3) ? -tau * (Txz * gr[0] + Tyz * gr[1] + Tzz * gr[2]) : 0.0f;
}

// accumulate p* = sum g, j = sum g e, Pi = sum g e e
template <int Q>
__device__ __forceinline__ void add_moments(int a, float v, float& p, float j[3], Stress& S) {
  using L = Lat<Q>;
  p += v;
  if (L::ex[a]) { j[0] += L::ex[a] * v; S.xx += v; }
  if (L::ey[a]) { j[1] += L::ey[a] * v; S.yy += v; }
  if (L::D == 3 && L::ez[a]) { j[2] += L::ez[a] * v; S.zz += v; }
  if (L::ex[a] && L::ey[a]) S.xy += (L::ex[a] * L::ey[a]) * v;
  if (L::D == 3 && L::ey[a] && L::ez[a]) S.yz += (L::ey[a] * L::ez[a]) * v;
  if (L::D == 3 && L::ex[a] && L::ez[a]) S.xz += (L::ex[a] * L::ez[a]) * v;
}

// everything both collisions need, from the stencil and the moments of g
struct NodeCtx {
  float phi, u[3], uu, om, tn[3];  // phase-field collision
  float p, f3r, F[3], s;           // hydrodynamic equilibrium, forcing, relaxation rate
  float cxx, cyy, czz, cxy, cyz, cxz;  // (1 - s) times the stress-projection coefficients
};

// Macroscopic update (Eqs. density_interpolation, chemical_potential,
// surface_tension_force, density_gradient_phase_field, relaxation_time,
// pressure_force, total_force, velocity_update) and the collision constants
// of the WMRT operator, or of the BGK operator (BGK).
template <int Q, bool BGK>
__device__ __forceinline__ void macro(const KParams& P, float phi, const float gr[3], float lap, float p,
                                      const float j[3], const Stress& S, const float up[3], NodeCtx& X) {
  constexpr int D = Lat<Q>::D;
  const float phc = P.clamp ? fminf(fmaxf(phi, 0.0f), 1.0f) : phi;
  const float rho = P.rho_l + phc * P.drho;
  const float inv_rho = 1.0f / rho;
  const float mu = P.beta4 * phi * (phi - 1.0f) * (phi - 0.5f) - P.kappa * lap;  // bulk term sign-corrected
  const float fb = rho - P.fb_rhol;
  float Fsb[3], grho[3];
  Fsb[0] = mu * gr[0] + fb * P.gx;
  Fsb[1] = mu * gr[1] + fb * P.gy;
  Fsb[2] = mu * gr[2] + fb * P.gz;
  grho[0] = P.drho * gr[0];
  grho[1] = P.drho * gr[1];
  grho[2] = P.drho * gr[2];
  const float tau = P.tau_l + phc * P.dtau;
  const float s = 1.0f / (tau + 0.5f);
  const float p3 = p * (1.0f / 3.0f);
  // velocity with the viscous force evaluated at the stored velocity
  float Fm[3];
  viscous_force<D, BGK>(S, p, up, tau, s, grho, Fm);
  float u[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) u[d] = j[d] + 0.5f * (Fsb[d] - p3 * grho[d] + Fm[d]) * inv_rho;
  if (D == 2) u[2] = 0.0f;
  // collision force with the viscous force re-evaluated at u^n
  float Fc[3];
  viscous_force<D, BGK>(S, p, u, tau, s, grho, Fc);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    X.u[d] = u[d];
    X.F[d] = Fsb[d] - p3 * grho[d] + Fc[d];
  }
  X.uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  X.phi = phi;
  X.p = p;
  X.s = s;
  X.f3r = 3.0f * inv_rho;
  // phase-field forcing direction (Eq. forcing_term)
  const float theta = (1.0f - 4.0f * (phi - 0.5f) * (phi - 0.5f)) * P.inv_xi;
  const float nrm = rsqrtf(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2] + 1e-24f);
  X.tn[0] = theta * gr[0] * nrm;
  X.tn[1] = theta * gr[1] * nrm;
  X.tn[2] = theta * gr[2] * nrm;
  X.om = P.omega_h;
  if (BGK) return;  // BGK relaxes every population at s: no projection
  // WMRT: only the deviatoric second moments of g - fbar, dev(Pi - u u), keep
  // a (1 - s) share; the projection coefficients follow
  const float dxx = S.xx - u[0] * u[0], dyy = S.yy - u[1] * u[1];
  const float dzz = (D == 3) ? S.zz - u[2] * u[2] : 0.0f;
  const float dxy = S.xy - u[0] * u[1];
  const float dyz = (D == 3) ? S.yz - u[1] * u[2] : 0.0f;
  const float dxz = (D == 3) ? S.xz - u[0] * u[2] : 0.0f;
  const float one_s = 1.0f - s;
  if (D == 3) {  // weighted basis: P y = 4.5 w_a (e e : dev)
    const float tr = (dxx + dyy + dzz) * (1.0f / 3.0f);
    X.cxx = 4.5f * one_s * (dxx - tr);
    X.cyy = 4.5f * one_s * (dyy - tr);
    X.czz = 4.5f * one_s * (dzz - tr);
    X.cxy = 9.0f * one_s * dxy;
    X.cyz = 9.0f * one_s * dyz;
    X.cxz = 9.0f * one_s * dxz;
  } else {  // plain orthogonal D2Q9 basis: P y = [(ex^2-ey^2)(dxx-dyy) + ex ey dxy] / 4
    X.cxx = 0.25f * one_s * (dxx - dyy);
    X.cyy = -X.cxx;
    X.czz = 0.0f;
    X.cxy = 0.25f * one_s * dxy;
    X.cyz = X.cxz = 0.0f;
  }
}

// post-collision h_a (Eqs. lbe_interface, forcing_term, equilibrium_with_force,
// equilibrium_function)
template <int Q>
__device__ __forceinline__ float h_post(const NodeCtx& X, int a, float ha) {
  using L = Lat<Q>;
  const float w = L::w[a];
  const float eu = L::ex[a] * X.u[0] + L::ey[a] * X.u[1] + L::ez[a] * X.u[2];
  const float heq = X.phi * w * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * X.uu);
  const float fphi = w * (L::ex[a] * X.tn[0] + L::ey[a] * X.tn[1] + L::ez[a] * X.tn[2]);
  return ha - X.om * (ha - heq + 0.5f * fphi) + fphi;
}

// post-collision g_a: f^eq + F_a/2 + (1 - s) P(g - fbar)_a, the closed form of
// Eqs. lbe_standard, mrt_collision, equilibrium_modified, force_term; BGK
// (Eq. bgk_collision): g_a - s (g_a - fbar_a) + F_a = (1 - s) g_a + s f^eq_a + (1 - s/2) F_a
template <int Q, bool BGK>
__device__ __forceinline__ float g_post(const NodeCtx& X, int a, float ga) {
  using L = Lat<Q>;
  const int ex = L::ex[a], ey = L::ey[a], ez = L::ez[a];
  const float w = L::w[a];
  const float eu = ex * X.u[0] + ey * X.u[1] + ez * X.u[2];
  const float feq = w * (X.p + 3.0f * eu + 4.5f * eu * eu - 1.5f * X.uu);
  const float Fa = w * X.f3r * (ex * X.F[0] + ey * X.F[1] + ez * X.F[2]);
  if (BGK) return (1.0f - X.s) * ga + X.s * feq + (1.0f - 0.5f * X.s) * Fa;
  float proj = 0.0f;
  if (ex) proj += X.cxx;
  if (ey) proj += X.cyy;
  if (ez) proj += X.czz;
  if (ex && ey) proj += (ex * ey) * X.cxy;
  if (ey && ez) proj += (ey * ez) * X.cyz;
  if (ex && ez) proj += (ex * ez) * X.cxz;
  if (L::D == 3) proj *= w;
  return feq + 0.5f * Fa + proj;
}

__device__ __forceinline__ void kahan_add(float v, float& s, float& c) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// stencil sums of phi (Eqs. gradient_phi, laplacian_phi; c = dx = 1)
template <int Q>
__device__ __forceinline__ void stencil_add(int a, float pn, float phi, float gr[3], float& lap) {
  using L = Lat<Q>;
  const float w = L::w[a];
  if (L::ex[a]) gr[0] += (w * L::ex[a]) * pn;
  if (L::ey[a]) gr[1] += (w * L::ey[a]) * pn;
  if (L::D == 3 && L::ez[a]) gr[2] += (w * L::ez[a]) * pn;
  lap += w * (pn - phi);
}

// Neighbour offsets of node c with periodic wrap (only valid where no
// non-periodic face is touched): n(c + e) = node + ox[ex+1] + oy[ey+1] + oz[ez+1].
struct Nbr {
  int node, ox[3], oy[3], oz[3];
  template <int Q>
  __device__ __forceinline__ int at(int a) const {
    return node + ox[Lat<Q>::ex[a] + 1] + oy[Lat<Q>::ey[a] + 1] + oz[Lat<Q>::ez[a] + 1];
  }
};

// Neighbour offsets of node c: periodic faces wrap; across a wall face the
// offset is clamped to the node itself (the ghost rule of the phase-field
// stencil, and the tangential neighbour of a reflected population).
__device__ __forceinline__ Nbr make_nbr(const KParams& P, const int c[3]) {
  Nbr n;
  n.node = node_of(P, c[0], c[1], c[2]);
  const int sxy = P.nx * P.ny;
  const bool px = P.bc[0] == BC_PERIODIC, py = P.bc[2] == BC_PERIODIC, pz = P.bc[4] == BC_PERIODIC;
  n.ox[0] = c[0] == 0 ? (px ? P.nx - 1 : 0) : -1;
  n.ox[1] = 0;
  n.ox[2] = c[0] == P.nx - 1 ? (px ? 1 - P.nx : 0) : 1;
  n.oy[0] = c[1] == 0 ? (py ? (P.ny - 1) * P.nx : 0) : -P.nx;
  n.oy[1] = 0;
  n.oy[2] = c[1] == P.ny - 1 ? (py ? (1 - P.ny) * P.nx : 0) : P.nx;
  n.oz[0] = c[2] == 0 ? (pz ? (P.nz - 1) * sxy : 0) : -sxy;
  n.oz[1] = 0;
  n.oz[2] = c[2] == P.nz - 1 ? (pz ? (1 - P.nz) * sxy : 0) : sxy;
  return n;
}

// Phase field of the stencil, from global memory (neighbour offsets) or from
// an LDS tile of three planes with a one-node halo (the marching kernel).
struct PhiGlobal {
  const __attribute__((address_space(1))) float* p;
  template <int Q>
  __device__ __forceinline__ float at(const Nbr& nb, int a) const {
    return p[a == 0 ? nb.node : nb.at<Q>(a)];
  }
};
struct PhiLds {
  const float* pl[3];  // planes z-1, z, z+1
  int li, W;           // this node's cell in a plane, row pitch of the tile
  template <int Q>
  __device__ __forceinline__ float at(const Nbr&, int a) const {
    return pl[Lat<Q>::ez[a] + 1][li + Lat<Q>::ey[a] * W + Lat<Q>::ex[a]];
  }
};

// Walls of the x axis are handled inside the tiled kernels: their nodes are
// one per row, so a separate face launch would read and write them one value
// per memory line.  Bit 0 (1) of the result: node c lies on the minus (plus)
// x face and that face is a wall.
__device__ __forceinline__ int wall_lane(const KParams& P, const int c[3]) {
  return ((c[0] == 0 ? 1 : 0) | (c[0] == P.nx - 1 ? 2 : 0)) & P.wbits;
}

// true if c + e_t lies beyond an x wall, for a node with wall bits `on`
template <int Q>
__device__ __forceinline__ bool wall_hit(int on, int t) {
  const int e = Lat<Q>::ex[t];
  return e != 0 && ((on >> (e > 0 ? 1 : 0)) & 1);
}

// Slot (population index, node) that receives post-collision population t
// of node nb.node -- the slot that t's opposite was read from -- and the node
// that reads the slot at the next step.  Even steps: pop[tbar][x]; odd steps:
// pop[t][x + e_t].  On an x-wall lane (WALL) a target beyond the wall becomes
// the x-reflected population of the tangential neighbour (free slip) or
// pop[tbar] of the node itself (no slip), as in the general path.
template <int Q, int ODD, bool WALL>
__device__ __forceinline__ void slot_of(const Nbr& nb, int on, int onns, int t, int& pop, int& nd, int& rdr) {
  rdr = nb.at<Q>(t);
  pop = ODD ? t : Lat<Q>::opp[t];
  nd = ODD ? rdr : nb.node;
  if (!WALL) return;
  if (ODD && wall_hit<Q>(on, t)) pop = reflect<Q>(t, 1);
  if (wall_hit<Q>(onns, t)) {
    rdr = nb.node;
    if (ODD) {
      pop = Lat<Q>::opp[t];
      nd = nb.node;
    }
  }
}

// true if the node touches a face whose boundary is not periodic
template <int Q>
__device__ __forceinline__ bool on_special_face(const KParams& P, const int c[3]) {
  bool s = false;
#pragma unroll
  for (int d = 0; d < Lat<Q>::D; ++d) {
    const int n = dim_of(P, d);
    s |= (c[d] == 0 && P.bc[2 * d] != BC_PERIODIC) || (c[d] == n - 1 && P.bc[2 * d + 1] != BC_PERIODIC);
  }
  return s;
}

// ---------------------------------------------------------------------------
// k_step: fused macroscopic update + both collisions + AA streaming
// ---------------------------------------------------------------------------

// Interior / periodic node: populations are consumed as they arrive, no
// per-direction arrays are held.  The h collision conserves sum_a h_a exactly
// (sum Gamma_a = 1, sum F^phi_a = 0); FP32 rounding (e.g. the FP32 weights
// sum to 1 + O(1e-8)) would leave a small systematic mass drift per step, so
// the node's mass is restored on the rest population with compensated sums
// (a zero correction in exact arithmetic).
template <int Q, int ST, int ODD, bool NT, bool WALL, bool BGK, class PhiSrc>
__device__ __forceinline__ void step_fast(const KParams& P, const KBufs& B, const int c[3], const PhiSrc& PS) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  using C = Codec<ST>;
  using Ty = typename C::T;
  const Nbr nb = make_nbr(P, c);
  const int node = nb.node;
  const int on = WALL ? wall_lane(P, c) : 0;
  const int onns = on & P.nsbits;
  const unsigned N = (unsigned)P.N;
  using GTy = __attribute__((address_space(1))) Ty;
  using GF = __attribute__((address_space(1))) float;
  GTy* Gp = (GTy*)B.g;  // loads and stores go through one pointer: in place
  GTy* Hp = (GTy*)B.h;
  GF* Uv = (GF*)B.u;

  const float phi = PS.template at<Q>(nb, 0);
  float gr[3] = {0.f, 0.f, 0.f}, lap = 0.f;
  float phn[Q];  // neighbours' phase field, kept: the 16-bit forms encode with the readers' one
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    phn[a] = PS.template at<Q>(nb, a);
    stencil_add<Q>(a, phn[a], phi, gr, lap);
  }
  gr[0] *= 3.0f;
  gr[1] *= 3.0f;
  gr[2] *= 3.0f;
  lap *= 6.0f;

  // Population a is read from the slot of abar (slot_of) and its
  // post-collision value goes to the slot abar was read from.  Slots are
  // addressed as a per-population base (uniform away from wall lanes) plus a
  // 32-bit node index.
  const size_t NN = (size_t)P.N;
  // On wall lanes the slot's population differs from the uniform one by at
  // most 3 (x reflection) or 1 (bounce-back), so the per-lane part stays a
  // signed 32-bit index (|index| < 4N < 2^31 for every admissible grid).
  auto sbase = [&](int t, int& idx, int& rdr) -> size_t {
    int pop, nd;
    slot_of<Q, ODD, WALL>(nb, on, onns, t, pop, nd, rdr);
    const int pop0 = ODD ? t : L::opp[t];
    idx = WALL ? nd + (pop - pop0) * (int)P.N : nd;
    return (size_t)pop0 * NN;
  };

  // hydrodynamic moments, opposite pairs summed and differenced (BGK keeps
  // the populations for the collision)
  float g0 = C::ld_g(Gp, (unsigned)node, L::w[0]);
  float gv[Q];
  float p = g0, j[3] = {0.f, 0.f, 0.f};
  Stress S = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const int b = L::opp[a];
    if (b < a) continue;
    int ia, ib;
    int ra, rb;
    const GTy* Ga = Gp + sbase(b, ia, ra);
    const GTy* Gb = Gp + sbase(a, ib, rb);
    const float ga = C::ld_g(Ga, ia, L::w[a]);
    const float gb = C::ld_g(Gb, ib, L::w[b]);
    if (BGK) {
      gv[a] = ga;
      gv[b] = gb;
    }
    const float s = ga + gb, d = ga - gb;
    p += s;
    if (L::ex[a]) { j[0] += L::ex[a] * d; S.xx += s; }
    if (L::ey[a]) { j[1] += L::ey[a] * d; S.yy += s; }
    if (D == 3 && L::ez[a]) { j[2] += L::ez[a] * d; S.zz += s; }
    if (L::ex[a] && L::ey[a]) S.xy += (L::ex[a] * L::ey[a]) * s;
    if (D == 3 && L::ey[a] && L::ez[a]) S.yz += (L::ey[a] * L::ez[a]) * s;
    if (D == 3 && L::ex[a] && L::ez[a]) S.xz += (L::ex[a] * L::ez[a]) * s;
  }
  float up[3];
  up[0] = Uv[node];
  up[1] = Uv[N + node];
  up[2] = (D == 3) ? Uv[2 * N + node] : 0.0f;
  NodeCtx X;
  macro<Q, BGK>(P, phi, gr, lap, p, j, S, up, X);
  Uv[node] = X.u[0];
  Uv[N + node] = X.u[1];
  if (D == 3) Uv[2 * N + node] = X.u[2];

  // per-node constants of the pair updates
  const float gA = X.p - 1.5f * X.uu;  // f^eq: w (gA + 4.5 eu^2 + 3 eu)
  const float hB = 1.0f - 1.5f * X.uu; // h^eq: phi w (hB + 4.5 eu^2 + 3 eu)
  const float hf = 0.5f * X.f3r;       // half of F_a / (w e.F)
  const float om = X.om;
  const float ref = (ST == 0) ? 0.0f : ((const GF*)B.ref)[node];

  // rest population
  const float h0 = C::ld_h(Hp, (unsigned)node, L::w[0], ref);
  {
    const float w = L::w[0];
    // e_0 = 0: no forcing, no stress projection
    const float g0p = BGK ? (1.0f - X.s) * g0 + X.s * (w * gA) : w * gA;
    C::template st_g<NT>(Gp, (unsigned)node, g0p, 1.0f / w);
  }
  const float d0 = om * (X.phi * L::w[0] * hB - h0);
  float dsum = d0;  // sum of the increments h+_a - h_a
  // momentum of the stored post-collision g, summed as stored; the axis
  // pairs come last and carry the momentum correction (below)
  float mom[3] = {0.f, 0.f, 0.f};

  // pairs (a, abar): even parts of the equilibria and of the stress
  // projection are shared, odd parts change sign.  Pairs are taken in
  // descending index order, so the axis pairs (1, 2), (3, 4), (5, 6) come
  // after every pair with a component along their axis.
#pragma unroll
  for (int k = Q - 1; k >= 1; --k) {
    const int a = k;
    const int b = L::opp[a];
    if (b < a) continue;
    const int ex = L::ex[a], ey = L::ey[a], ez = L::ez[a];
    const float w = L::w[a];
    int ia, ib;
    int rdr_b, rdr_a;  // readers of the slots of a's and b's post-collision values
    const size_t oa = sbase(b, ia, rdr_b);  // a is read here, b's post value goes here
    const size_t ob = sbase(a, ib, rdr_a);
    GTy* Ha = Hp + oa;
    GTy* Hb = Hp + ob;
    GTy* Ga = Gp + oa;
    GTy* Gb = Gp + ob;
    const float ha = C::ld_h(Ha, ia, w, ref);
    const float hb = C::ld_h(Hb, ib, w, ref);
    const float eu = ex * X.u[0] + ey * X.u[1] + ez * X.u[2];
    const float eu2 = eu * eu;
    // hydrodynamic set
    const float eF = ex * X.F[0] + ey * X.F[1] + ez * X.F[2];
    float va, vb;  // post-collision a (stored where b was read) and b
    if (BGK) {  // (1 - s) g + s f^eq + (1 - s/2) F_a, even and odd parts
      const float sr = X.s;
      const float gsym = sr * w * (gA + 4.5f * eu2);
      const float ganti = w * (sr * 3.0f * eu + (2.0f - sr) * hf * eF);
      va = (1.0f - sr) * gv[a] + gsym + ganti;
      vb = (1.0f - sr) * gv[b] + gsym - ganti;
    } else {
      float proj = 0.0f;
      if (ex) proj += X.cxx;
      if (ey) proj += X.cyy;
      if (ez) proj += X.czz;
      if (ex && ey) proj += (ex * ey) * X.cxy;
      if (ey && ez) proj += (ey * ez) * X.cyz;
      if (ex && ez) proj += (ex * ez) * X.cxz;
      if (D == 2) proj *= (1.0f / w);  // the D2Q9 projection is not weighted
      const float gsym = w * (gA + 4.5f * eu2 + proj);
      const float ganti = w * (3.0f * eu + hf * eF);
      va = gsym + ganti;
      vb = gsym - ganti;
    }
    const float dv = va - vb;
    if (ex) mom[0] += ex * dv;
    if (ey) mom[1] += ey * dv;
    if (ez) mom[2] += ez * dv;
    const int nax = (ex != 0) + (ey != 0) + (ez != 0);
    if (nax == 1) {
      // The post-collision momentum is u + F / (2 rho) (WMRT) or
      // (1 - s) j + s u + (1 - s/2) F / rho (BGK) in exact arithmetic.  With
      // the FP32 weights the stored values carry it scaled by 1 + O(1e-8)
      // with a fixed sign (6 (w_1 + 4 w_2) - 1 = 7.5e-9 in D3Q19), a drift
      // that compounds over the steps; the axis pair of each direction, the
      // last pair with a component along it, takes the difference (+c/2 on
      // a, -c/2 on abar: mass and second moments unchanged).
      const int d = ex ? 0 : (ey ? 1 : 2);
      const int sg = ex + ey + ez;  // +1: a points along +d
      const float target = BGK ? (1.0f - X.s) * j[d] + X.s * X.u[d] +
                                     (1.0f - 0.5f * X.s) * X.F[d] * X.f3r * (1.0f / 3.0f)
                               : X.u[d] + X.F[d] * X.f3r * (1.0f / 6.0f);
      const float c = 0.5f * (float)sg * (target - mom[d]);
      va += c;
      vb -= c;
    }
    C::template st_g<NT>(Gb, ib, va, 1.0f / w);  // a goes where b was read
    C::template st_g<NT>(Ga, ia, vb, 1.0f / w);
    // phase-field set
    const float pw = X.phi * w;
    const float hsym = pw * (hB + 4.5f * eu2);
    const float fphi = w * (ex * X.tn[0] + ey * X.tn[1] + ez * X.tn[2]);
    const float hanti = pw * (3.0f * eu) - 0.5f * fphi;  // odd part of h^eq - F^phi/2
    const float da = om * (hsym + hanti - ha) + fphi;
    const float db = om * (hsym - hanti - hb) - fphi;
    dsum += da + db;
    // readers' phase field: the stencil's neighbour in direction a (b), the
    // clamped one at a free-slip x wall, or the node itself where a no-slip
    // x wall sends the value back (slot_of)
    const float wra = (ST == 0) ? 0.0f : ((WALL && wall_hit<Q>(onns, a)) ? phi : phn[a]);
    const float wrb = (ST == 0) ? 0.0f : ((WALL && wall_hit<Q>(onns, b)) ? phi : phn[b]);
    C::template st_h<NT>(Hb, ib, ha + da, 1.0f / w, wra);
    C::template st_h<NT>(Ha, ia, hb + db, 1.0f / w, wrb);
  }
  // sum_a (h+_a - h_a) vanishes in exact arithmetic (sum Gamma_a = 1, sum
  // F^phi_a = 0); FP32 leaves O(1e-8) per node per step with a systematic
  // part (the FP32 weights sum to 1 + O(1e-8)), so it is removed on the rest
  // population to keep the node's mass.
  C::template st_h<NT>(Hp, (unsigned)node, h0 + (d0 - dsum), 1.0f / L::w[0], (ST == 0) ? 0.0f : phi);
}

// Nodes on wall, inlet or outlet faces: general slot resolution with arrays.
template <int Q, int ST, int ODD, bool NT, bool BGK>
__device__ __forceinline__ void step_general(const KParams& P, const KBufs& B, const int c[3]) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  using C = Codec<ST>;
  using Ty = typename C::T;
  const int node = node_of(P, c[0], c[1], c[2]);
  const size_t N = (size_t)P.N;

  const float phi = B.phi[node];
  float gr[3] = {0.f, 0.f, 0.f}, lap = 0.f;
#pragma unroll
  for (int a = 1; a < Q; ++a) stencil_add<Q>(a, phi_nb<Q>(P, B.phi, c, a), phi, gr, lap);
  gr[0] *= 3.0f;
  gr[1] *= 3.0f;
  gr[2] *= 3.0f;
  lap *= 6.0f;

  float h[Q], g[Q];
  load_node<Q, ST, ODD, true>(P, B, c, h, g);
  float p = 0.f, j[3] = {0.f, 0.f, 0.f};
  Stress S = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < Q; ++a) add_moments<Q>(a, g[a], p, j, S);
  float up[3];
  up[0] = B.u[node];
  up[1] = B.u[N + node];
  up[2] = (D == 3) ? B.u[2 * N + node] : 0.0f;
  NodeCtx X;
  macro<Q, BGK>(P, phi, gr, lap, p, j, S, up, X);
  B.u[node] = X.u[0];
  B.u[N + node] = X.u[1];
  if (D == 3) B.u[2 * N + node] = X.u[2];

  Ty* Gw = (Ty*)B.g;
  // post-collision g with the momentum correction of the fast path: the
  // difference between the exact post-collision momentum and the one the
  // FP32 values carry goes to the axis pairs
  float gq[Q], mom[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    gq[a] = g_post<Q, BGK>(X, a, g[a]);
    if (L::ex[a]) mom[0] += L::ex[a] * gq[a];
    if (L::ey[a]) mom[1] += L::ey[a] * gq[a];
    if (D == 3 && L::ez[a]) mom[2] += L::ez[a] * gq[a];
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const float target = BGK ? (1.0f - X.s) * j[d] + X.s * X.u[d] + (1.0f - 0.5f * X.s) * X.F[d] * X.f3r * (1.0f / 3.0f)
                             : X.u[d] + X.F[d] * X.f3r * (1.0f / 6.0f);
    const float cc = 0.5f * (target - mom[d]);
    const int ap = d == 0 ? find_vel<Q>(1, 0, 0) : (d == 1 ? find_vel<Q>(0, 1, 0) : find_vel<Q>(0, 0, 1));
    gq[ap] += cc;
    gq[L::opp[ap]] -= cc;
  }
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int sp, sn;
    if (resolve_dst<Q, ODD>(P, c, a, sp, sn))
      C::template st_g<NT>(Gw, (size_t)sp * N + sn, gq[a], 1.0f / L::w[a]);
  }
  float pre_s = 0.f, pre_c = 0.f, post_s = 0.f, post_c = 0.f;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    kahan_add(h[a], pre_s, pre_c);
    h[a] = h_post<Q>(X, a, h[a]);
    kahan_add(h[a], post_s, post_c);
  }
  h[0] += (pre_s - post_s) - (pre_c - post_c);
  Ty* Hw = (Ty*)B.h;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int sp, sn;
    if (!resolve_dst<Q, ODD>(P, c, a, sp, sn)) continue;
    float ref = 0.0f;
    if (ST != 0) {  // encode relative to the reader's phase field
      int tn;
      stream_target<Q>(P, c, a, tn);
      ref = B.phi[tn];
    }
    C::template st_h<NT>(Hw, (size_t)sp * N + sn, h[a], 1.0f / L::w[a], ref);
  }
}

// Tiled box: the whole grid less the face layers of non-periodic y and z axes
// (x walls stay in the box as wall lanes).
struct Box {
  int x0, y0, z0, nx, ny, nz;  // origin and extent
};

// node of thread tid in tile L of the box (x fastest, then y, then z)
__device__ __forceinline__ bool tile_node(const Box& X, const Tiling& T, int L, int tid, int c[3]) {
  const int tx = L % T.ntx;
  const int r = L / T.ntx;
  const int ty = r % T.nty;
  const int lx = tx * T.bx + tid % T.bx;
  const int ly = ty * T.by + tid / T.bx;
  c[0] = X.x0 + lx;
  c[1] = X.y0 + ly;
  c[2] = X.z0 + r / T.nty;
  return lx < X.nx && ly < X.ny;
}

__device__ __forceinline__ bool box_coords(const Box& X, const Tiling& T, int c[3]) {
  return tile_node(X, T, xcd_remap(blockIdx.x, gridDim.x), (int)threadIdx.x, c);
}

// Face layers (general path), enumerated without overlap and with x fastest
// so that a wave covers contiguous nodes: in 3D the y = 0 and y = ny-1 rows
// of the box's z range (non-periodic y), then the two planes of the last
// axis (non-periodic z in 3D, y in 2D), minus side first.
struct Faces {
  int n1, n2;    // nodes of the y rows (3D) and of the last-axis planes
  int z0, nzb;   // z range of the y rows
};

template <int Q>
__device__ __forceinline__ void face_coords(const KParams& P, const Faces& F, int t, int c[3]) {
  if (Lat<Q>::D == 3 && t < F.n1) {
    const int half = F.n1 >> 1;
    const int side = t >= half ? 1 : 0;
    const int r = t - side * half;
    c[0] = r % P.nx;
    c[1] = side ? P.ny - 1 : 0;
    c[2] = F.z0 + r / P.nx;
    return;
  }
  t -= F.n1;
  const int side = t >= P.plane ? 1 : 0;
  const int r = t - side * P.plane;
  if (Lat<Q>::D == 3) {
    c[0] = r % P.nx;
    c[1] = r / P.nx;
    c[2] = side ? P.nz - 1 : 0;
  } else {
    c[0] = r;
    c[1] = side ? P.ny - 1 : 0;
    c[2] = 0;
  }
}

// ---------------------------------------------------------------------------
// phase field phi = sum_a h_a of the current state (Eq. phase_field_variable),
// compensated sum; interior nodes and face-layer nodes
// ---------------------------------------------------------------------------
template <int Q, int ST, int ODD, bool WALL>
__device__ __forceinline__ void phi_fast(const KParams& P, const KBufs& B, const int c[3]) {
  using L = Lat<Q>;
  using C = Codec<ST>;
  using Ty = typename C::T;
  const Nbr nb = make_nbr(P, c);
  const int node = nb.node;
  const int on = WALL ? wall_lane(P, c) : 0;
  const int onns = on & P.nsbits;
  const size_t NN = (size_t)P.N;
  using GTy = __attribute__((address_space(1))) Ty;
  using GF = __attribute__((address_space(1))) float;
  const GTy* Hp = (const GTy*)B.h;
  const float ref = (ST == 0) ? 0.0f : ((const GF*)B.ref)[node];
  float s = 0.0f, cc = 0.0f;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int pop, nd, rdr;
    const int t = L::opp[a];  // a is read from the slot of abar
    slot_of<Q, ODD, WALL>(nb, on, onns, t, pop, nd, rdr);
    const int pop0 = ODD ? t : a;
    const int idx = WALL ? nd + (pop - pop0) * P.N : nd;
    kahan_add(C::ld_h(Hp + (size_t)pop0 * NN, idx, L::w[a], ref), s, cc);
  }
  ((GF*)B.phi_out)[node] = s - cc;
}

template <int Q, int ST, int ODD>
__device__ __forceinline__ void phi_general(const KParams& P, const KBufs& B, const int c[3]) {
  const int node = node_of(P, c[0], c[1], c[2]);
  float phi;
  if (is_inlet_node<Q>(P, c)) {
    float p0, p1;
    inlet_tangential<Q>(c, p0, p1);
    phi = inlet_psi(P, p0, p1);  // sum_a h_a = phi_in exactly after the inlet condition
  } else {
    float h[Q], g[1], lo;
    load_node<Q, ST, ODD, false>(P, B, c, h, g);
    kahan_sum<Q>(h, phi, lo);
    phi += lo;
  }
  B.phi_out[node] = phi;
}

// ---------------------------------------------------------------------------
// k_outlet: convective outflow (appendix B) after the step of parity ODD
// ---------------------------------------------------------------------------
template <int Q, int ST, int ODD>
__device__ __forceinline__ void outlet_node(const KParams& P, const KBufs& B, int pi, const float* uplane) {
  constexpr int AX = Lat<Q>::AX;
  int c[3];
  if (Lat<Q>::D == 3) {
    c[0] = pi % P.nx;
    c[1] = pi / P.nx;
    c[2] = P.nz - 2;
  } else {
    c[0] = pi;
    c[1] = P.ny - 2;
    c[2] = 0;
  }
  // populations streamed into the layer N-1 (read as the next step will)
  float h[Q], g[Q];
  load_node<Q, ST, !ODD, true>(P, B, c, h, g);
  const int node = node_of(P, c[0], c[1], c[2]);
  // local option: the outward velocity of this node; plane options: the
  // clipped maximum or average over the layer, from k_outlet_speed
  const float U = P.outlet_mode == 0 ? fmaxf(B.u[(size_t)AX * P.N + node], 0.0f) : *uplane;
  const float inv = 1.0f / (1.0f + U);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    float* oh = B.obuf + (size_t)a * P.plane + pi;
    float* og = B.obuf + (size_t)(Q + a) * P.plane + pi;
    *oh = (*oh + U * h[a]) * inv;
    *og = (*og + U * g[a]) * inv;
  }
}

// ---------------------------------------------------------------------------
// Launches over a table of domains (one domain for a single simulation, many
// for the batched form): every domain has its own parameters and buffers.
// ---------------------------------------------------------------------------
struct DomDev {
  KParams K;
  KBufs B[2];   // buffers of a step of parity 0 / 1
  KBufs Bo[2];  // buffers of the outlet update after a step of parity 0 / 1
  Box X;
  Faces F;
  int ntx, nty, ntiles;     // interior tiling
  int tile_base, face_base, plane_base;
  int task_base;            // first z-marching task of the domain (D3Q19)
  float* uplane;            // convective velocity of the plane options (one float)
};

// Persistent, chunked launch over the tile list of all domains: each block
// walks a contiguous chunk of tiles (contiguous per XCD after the remap), so
// neighbouring tiles of one domain share an L2.
template <int Q, int ST, int ODD, bool NT, bool PHI, bool WALL, bool BGK>
__global__ __launch_bounds__(512) void kb_interior(const DomDev* __restrict__ D, const int* __restrict__ tile_dom,
                                                   int ntiles, int chunk, int bx, int by) {
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int t0 = L * chunk;
  const int t1 = min(t0 + chunk, ntiles);
  for (int t = t0; t < t1; ++t) {
    const int d = tile_dom ? tile_dom[t] : 0;
    const DomDev& dm = D[d];
    Tiling T;
    T.bx = bx;
    T.by = by;
    T.ntx = dm.ntx;
    T.nty = dm.nty;
    T.ntiles = dm.ntiles;
    int c[3];
    if (!tile_node(dm.X, T, t - dm.tile_base, (int)threadIdx.x, c)) continue;
    if (PHI)
      phi_fast<Q, ST, ODD, WALL>(dm.K, dm.B[ODD], c);
    else
      step_fast<Q, ST, ODD, NT, WALL, BGK>(dm.K, dm.B[ODD], c,
                                           PhiGlobal{(const __attribute__((address_space(1))) float*)dm.B[ODD].phi});
  }
}

// index on an axis of n nodes for a stencil cell: periodic axes wrap, others
// clamp to the face node (the ghost rule of the phase-field stencil; cells
// beyond the box's last partial tile stay in bounds and are read by no node)
__device__ __forceinline__ int cell_axis(int v, int n, bool periodic) {
  if (periodic) return ((v % n) + n) % n;
  return min(max(v, 0), n - 1);
}

// Interior step of a D3Q19 domain marching along z.  A task is one tile
// (bx x by nodes) of a domain's box over a chunk of zc planes; the phase field
// of the tile and its one-node halo is staged in an LDS ring of five planes,
// one plane loaded per plane advanced (one barrier per plane), and the
// stencil reads it there instead of 19 global loads per node.  Tasks are
// numbered tile-fastest within each z-chunk, and each persistent block walks
// a contiguous chunk of them (contiguous per XCD after the remap).
template <int ST, int ODD, bool NT, bool WALL, bool BGK>
__global__ __launch_bounds__(512) void kb_march(const DomDev* __restrict__ D, const int* __restrict__ task_dom,
                                                int ntasks, int chunk, int bx, int by, int zc) {
  extern __shared__ float ring[];
  const int W = bx + 2, PL = W * (by + 2);
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int t0 = L * chunk;
  const int t1 = min(t0 + chunk, ntasks);
  const int tid = (int)threadIdx.x, nth = (int)blockDim.x;
  const int i = tid % bx, j = tid / bx;
  for (int t = t0; t < t1; ++t) {
    const int d = task_dom ? task_dom[t] : 0;
    const DomDev& dm = D[d];
    const KParams& P = dm.K;
    const int nxy = dm.ntx * dm.nty;
    const int lt = t - dm.task_base;
    const int tile = lt % nxy, zci = lt / nxy;
    const int gx0 = dm.X.x0 + (tile % dm.ntx) * bx, gy0 = dm.X.y0 + (tile / dm.ntx) * by;
    const int zb = dm.X.z0 + zci * zc, ze = min(zb + zc, dm.X.z0 + dm.X.nz);
    const bool px = P.bc[0] == BC_PERIODIC, py = P.bc[2] == BC_PERIODIC, pz = P.bc[4] == BC_PERIODIC;
    const __attribute__((address_space(1))) float* Phi =
        (const __attribute__((address_space(1))) float*)dm.B[ODD].phi;
    auto load_plane = [&](int z) {  // plane z into its ring slot
      float* dst = ring + ((z - zb + 1) % 5) * PL;
      const int zr = cell_axis(z, P.nz, pz);
      for (int k = tid; k < PL; k += nth) {
        const int x = cell_axis(gx0 + k % W - 1, P.nx, px);
        const int y = cell_axis(gy0 + k / W - 1, P.ny, py);
        dst[k] = Phi[node_of(P, x, y, zr)];
      }
    };
    __syncthreads();  // the previous task's last plane has been read
    load_plane(zb - 1);
    load_plane(zb);
    load_plane(zb + 1);
    const bool valid = gx0 + i < dm.X.x0 + dm.X.nx && gy0 + j < dm.X.y0 + dm.X.ny;
    for (int z = zb; z < ze; ++z) {
      if (z + 2 <= ze) load_plane(z + 2);
      __syncthreads();
      if (valid) {
        const int c[3] = {gx0 + i, gy0 + j, z};
        const int m = z - zb + 1;  // ring index of plane z
        PhiLds PS;
        PS.pl[0] = ring + ((m + 4) % 5) * PL;
        PS.pl[1] = ring + (m % 5) * PL;
        PS.pl[2] = ring + ((m + 1) % 5) * PL;
        PS.li = (j + 1) * W + (i + 1);
        PS.W = W;
        step_fast<19, ST, ODD, NT, WALL, BGK>(P, dm.B[ODD], c, PS);
      }
    }
  }
}

// domain of flat index t given per-domain bases (ascending)
template <int WHICH>
__device__ __forceinline__ int find_dom(const DomDev* __restrict__ D, int ndom, int t) {
  int lo = 0, hi = ndom - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int base = WHICH == 0 ? D[mid].face_base : D[mid].plane_base;
    if (base <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int Q, int ST, int ODD, bool NT, bool PHI, bool BGK>
__global__ __launch_bounds__(256) void kb_faces(const DomDev* __restrict__ D, int ndom, int nface) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nface) return;
  const int d = find_dom<0>(D, ndom, t);
  const DomDev& dm = D[d];
  int c[3];
  face_coords<Q>(dm.K, dm.F, t - dm.face_base, c);
  if (PHI)
    phi_general<Q, ST, ODD>(dm.K, dm.B[ODD], c);
  else
    step_general<Q, ST, ODD, NT, BGK>(dm.K, dm.B[ODD], c);
}

template <int Q, int ST, int ODD>
__global__ __launch_bounds__(256) void kb_outlet(const DomDev* __restrict__ D, int ndom, int nplane) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nplane) return;
  const int d = find_dom<1>(D, ndom, t);
  const DomDev& dm = D[d];
  if (!dm.K.has_outlet) return;
  outlet_node<Q, ST, ODD>(dm.K, dm.Bo[ODD], t - dm.plane_base, dm.uplane);
}

// per-plane count of nodes with phi > threshold along the streamwise axis
// (one block per plane); used for the intact-length diagnostic
__global__ __launch_bounds__(256) void k_plane_count(const float* __restrict__ phi, int plane, int nplanes,
                                                     float thr, int* __restrict__ count) {
  __shared__ int sc[256];
  const int z = blockIdx.x;
  if (z >= nplanes) return;
  int n = 0;
  for (int i = threadIdx.x; i < plane; i += blockDim.x) n += phi[(size_t)z * plane + i] > thr ? 1 : 0;
  sc[threadIdx.x] = n;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sc[threadIdx.x] += sc[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[z] = sc[0];
}

// ---------------------------------------------------------------------------
// initial state, export, import, fields, reductions
// ---------------------------------------------------------------------------

// canonical (even-parity) initial populations from phi0, u0; the 16-bit
// reference of a canonical slot is phi0 of its own node (its reader).
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_init(KParams P, KBufs B, const float* __restrict__ phi0,
                                              const float* __restrict__ u0, Tiling T) {
  using L = Lat<Q>;
  using C = Codec<ST>;
  using Ty = typename C::T;
  int c[3];
  if (!tile_coords(P, T, c)) return;
  const int node = node_of(P, c[0], c[1], c[2]);
  const size_t N = (size_t)P.N;
  const float phi = phi0[node];
  float gr[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const float pn = phi_nb<Q>(P, phi0, c, a);
    gr[0] += (L::w[a] * L::ex[a]) * pn;
    gr[1] += (L::w[a] * L::ey[a]) * pn;
    gr[2] += (L::w[a] * L::ez[a]) * pn;
  }
  gr[0] *= 3.0f;
  gr[1] *= 3.0f;
  gr[2] *= 3.0f;
  float u[3] = {0.f, 0.f, 0.f};
  if (u0) {
    u[0] = u0[node];
    u[1] = u0[N + node];
    u[2] = (L::D == 3) ? u0[2 * N + node] : 0.0f;
  }
  B.u[node] = u[0];
  B.u[N + node] = u[1];
  B.u[2 * N + node] = u[2];
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const float theta = (1.0f - 4.0f * (phi - 0.5f) * (phi - 0.5f)) * P.inv_xi;
  const float nrm = rsqrtf(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2] + 1e-24f);
  const bool outlet = is_outlet_node<Q>(P, c);
  const int pi = plane_index<Q>(P, c);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const float w = L::w[a];
    const float eu = L::ex[a] * u[0] + L::ey[a] * u[1] + L::ez[a] * u[2];
    const float G1 = 1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;
    const float fphi = theta * w * (L::ex[a] * gr[0] + L::ey[a] * gr[1] + L::ez[a] * gr[2]) * nrm;
    const float hv = phi * w * G1 - 0.5f * fphi;
    const float gv = w * (3.0f * eu + 4.5f * eu * eu - 1.5f * uu);
    if (outlet) {
      B.obuf[(size_t)a * P.plane + pi] = hv;
      B.obuf[(size_t)(Q + a) * P.plane + pi] = gv;
    }
    int sp, sn, src;
    if (resolve_src<Q, 0>(P, c, a, sp, sn, src)) {
      C::st_h((Ty*)B.h, (size_t)sp * N + sn, hv, 1.0f / w, (ST == 0) ? 0.0f : phi);
      C::st_g((Ty*)B.g, (size_t)sp * N + sn, gv, 1.0f / w);
    }
  }
}

template <int Q, int ST, int ODD>
__global__ __launch_bounds__(256) void k_export(KParams P, KBufs B, float* __restrict__ ho,
                                                float* __restrict__ go, float* __restrict__ uo, Tiling T) {
  int c[3];
  if (!tile_coords(P, T, c)) return;
  const int node = node_of(P, c[0], c[1], c[2]);
  const size_t N = (size_t)P.N;
  float h[Q], g[Q];
  load_node<Q, ST, ODD, true>(P, B, c, h, g);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    if (ho) ho[(size_t)a * N + node] = h[a];
    if (go) go[(size_t)a * N + node] = g[a];
  }
  if (uo)
    for (int d = 0; d < 3; ++d) uo[(size_t)d * N + node] = B.u[(size_t)d * N + node];
}

// import, pass 1: reference phase field sum_a h_a of the canonical input
template <int Q>
__global__ __launch_bounds__(256) void k_import_ref(KParams P, const float* __restrict__ hi,
                                                    float* __restrict__ ref, Tiling T) {
  int c[3];
  if (!tile_coords(P, T, c)) return;
  const int node = node_of(P, c[0], c[1], c[2]);
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < Q; ++a) s += hi[(size_t)a * P.N + node];
  ref[node] = s;
}

// import, pass 2: store canonical populations in even-parity slots
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_import(KParams P, KBufs B, const float* __restrict__ hi,
                                                const float* __restrict__ gi, const float* __restrict__ ui,
                                                Tiling T) {
  using C = Codec<ST>;
  using Ty = typename C::T;
  int c[3];
  if (!tile_coords(P, T, c)) return;
  const int node = node_of(P, c[0], c[1], c[2]);
  const size_t N = (size_t)P.N;
  const bool outlet = is_outlet_node<Q>(P, c);
  const int pi = plane_index<Q>(P, c);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const float hv = hi[(size_t)a * N + node], gv = gi[(size_t)a * N + node];
    if (outlet) {
      B.obuf[(size_t)a * P.plane + pi] = hv;
      B.obuf[(size_t)(Q + a) * P.plane + pi] = gv;
    }
    int sp, sn, src;
    if (resolve_src<Q, 0>(P, c, a, sp, sn, src)) {
      const float w = Lat<Q>::w[a];
      C::st_h((Ty*)B.h, (size_t)sp * N + sn, hv, 1.0f / w, (ST == 0) ? 0.0f : B.ref[node]);
      C::st_g((Ty*)B.g, (size_t)sp * N + sn, gv, 1.0f / w);
    }
  }
  for (int d = 0; d < 3; ++d) B.u[(size_t)d * N + node] = ui[(size_t)d * N + node];
}

// p = p* rho cs^2 of the current state (phi from the current phase field)
template <int Q, int ST, int ODD>
__global__ __launch_bounds__(256) void k_pressure(KParams P, KBufs B, float* __restrict__ po, Tiling T) {
  int c[3];
  if (!tile_coords(P, T, c)) return;
  const int node = node_of(P, c[0], c[1], c[2]);
  float h[Q], g[Q];
  load_node<Q, ST, ODD, true>(P, B, c, h, g);
  float ps = 0.f, ph = 0.f;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    ps += g[a];
    ph += h[a];
  }
  const float phc = P.clamp ? fminf(fmaxf(ph, 0.0f), 1.0f) : ph;
  po[node] = ps * (P.rho_l + phc * P.drho) * (1.0f / 3.0f);
}

// FP64 sums of phi and 0.5 rho |u|^2: per-block partials in a fixed order
// FP64 sum over the 64 lanes of a wave (xor butterfly); every lane ends with
// a sum, and callers take lane 0's, whose order of additions is fixed.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of phi and of 0.5 rho |u|^2 per domain, in FP64: block b takes part
// (b % ppd) of domain (b / ppd), each thread a strided run of nodes, then a
// wave reduction and a fixed-order sum of the block's four waves; part[2b],
// part[2b + 1] receive the block's sums.  Deterministic for a given ppd.
template <int PAR>
__global__ __launch_bounds__(256) void k_reduce_partial(const DomDev* __restrict__ D, int ppd,
                                                        double* __restrict__ part) {
  const int d = blockIdx.x / ppd, j = blockIdx.x % ppd;
  const KParams& P = D[d].K;
  const float* __restrict__ phi = D[d].B[PAR].phi;
  const float* __restrict__ u = D[d].B[PAR].u;
  const size_t N = (size_t)P.N;
  const double rho_l = P.rho_l, drho = P.drho;
  const int clamp = P.clamp;
  double m = 0.0, k = 0.0;
  for (size_t i = (size_t)j * 256 + threadIdx.x; i < N; i += (size_t)ppd * 256) {
    const double ph = phi[i];
    const double phc = clamp ? fmin(fmax(ph, 0.0), 1.0) : ph;
    const double rho = rho_l + phc * drho;
    const double ux = u[i], uy = u[N + i], uz = u[2 * N + i];
    m += ph;
    k += 0.5 * rho * (ux * ux + uy * uy + uz * uz);
  }
  m = wave_sum(m);
  k = wave_sum(k);
  __shared__ double sm[4], sk[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[w] = m;
    sk[w] = k;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
    part[2 * blockIdx.x + 1] = ((sk[0] + sk[1]) + sk[2]) + sk[3];
  }
}

// One block per domain: the domain's ppd partials summed in a fixed order
// (strided per thread, wave reduction, the four waves in order) into
// out[2d] (sum phi) and out[2d + 1] (kinetic energy).
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ part, int ppd,
                                                      double* __restrict__ out) {
  const double* p = part + 2 * (size_t)blockIdx.x * ppd;
  double m = 0.0, k = 0.0;
  for (int i = threadIdx.x; i < ppd; i += 256) {
    m += p[2 * i];
    k += p[2 * i + 1];
  }
  m = wave_sum(m);
  k = wave_sum(k);
  __shared__ double sm[4], sk[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[w] = m;
    sk[w] = k;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
    out[2 * blockIdx.x + 1] = ((sk[0] + sk[1]) + sk[2]) + sk[3];
  }
}

// Convective velocity of the plane options (appendix B: U_max, U_ave): the
// outward normal velocity of the latest macroscopic update over the layer
// next to the outlet, its maximum or its average, clipped at zero.  One
// block per domain; the average is an FP64 sum in a fixed order.
template <int Q>
__global__ __launch_bounds__(256) void k_outlet_speed(const DomDev* __restrict__ D) {
  constexpr int AX = Lat<Q>::AX;
  const DomDev& dm = D[blockIdx.x];
  const KParams& P = dm.K;
  if (!P.has_outlet || P.outlet_mode == 0) return;
  const float* u = dm.B[0].u + (size_t)AX * P.N;
  const size_t base = (size_t)P.plane * (size_t)((AX == 2 ? P.nz : P.ny) - 2);
  float mx = -3.0e38f;
  double sum = 0.0;
  for (int i = threadIdx.x; i < P.plane; i += 256) {
    const float v = u[base + i];
    mx = fmaxf(mx, v);
    sum += (double)v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  sum = wave_sum(sum);
  __shared__ float smx[4];
  __shared__ double ssum[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smx[w] = mx;
    ssum[w] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(smx[0], smx[1]), fmaxf(smx[2], smx[3]));
    const double s = ((ssum[0] + ssum[1]) + ssum[2]) + ssum[3];
    const float U = P.outlet_mode == 1 ? m : (float)(s / (double)P.plane);
    *dm.uplane = fmaxf(U, 0.0f);
  }
}

}  // namespace lbm
