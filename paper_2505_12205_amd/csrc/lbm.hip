// lbm.hip -- host runtime and C ABI (include/lbm.h) of the gfx950
// phase-field lattice Boltzmann library.
//
// A simulation and a batch step through the same kernels: the launches run
// over a device table of domains (one entry for a simulation, many for a
// batch), so a domain advances bit for bit the same way in both.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lbm.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Capacity, in pairs of doubles, of the reduction partials of one launch.
constexpr int kReduceMaxParts = 16384;

}  // namespace

// Partial sums of the allocation-free batch reduction
// (lbm_batch_reduce_noalloc): kReduceMaxParts pairs of doubles, 256 KiB on
// each GPU the library runs on, held until the process ends.  Every call on a
// GPU shares that GPU's copy, so reductions that overlap on one GPU race.
static __device__ __align__(256) double scratch[2 * kReduceMaxParts];

namespace {

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;  // device address of `scratch`, per device ordinal

// Device address of the static scratch array on the current device, looked
// up once per device (host code must not pass the array's name to a kernel).
int scratch_on_current_device(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return LBM_OK;
}



struct Layout {
  size_t h, g, u, phi0, phi1, obuf, total;
};

int pop_size(int storage) { return storage == LBM_FP32 ? 4 : 2; }
int axis_of(int lattice) { return lattice == LBM_D2Q9 ? 1 : 2; }
int plane_of(const lbm_params& p) { return p.lattice == LBM_D2Q9 ? p.nx : p.nx * p.ny; }

bool has_bc(const lbm_params& p, int bc) {
  for (int f = 0; f < 6; ++f)
    if (p.bc[f] == bc) return true;
  return false;
}

int validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "null parameters");
  if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19) return fail(LBM_EINVAL, "lattice must be 9 or 19");
  if (p->nx < 2 || p->ny < 2 || p->nz < 1) return fail(LBM_EINVAL, "grid too small");
  if (p->lattice == LBM_D2Q9 && p->nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz = 1");
  if (p->lattice == LBM_D3Q19 && p->nz < 2) return fail(LBM_EINVAL, "D3Q19 needs nz >= 2");
  const double nodes = (double)p->nx * p->ny * p->nz;
  if (nodes >= 2147483647.0 / 4) return fail(LBM_EINVAL, "grid too large for one domain");
  if (!(p->tau_h > -0.5) || !(p->tau_l > -0.5)) return fail(LBM_EINVAL, "tau must exceed -1/2");
  if (!(p->xi > 0.0)) return fail(LBM_EINVAL, "xi must be positive");
  if (!(p->rho_l > 0.0) || !(p->rho_h > 0.0)) return fail(LBM_EINVAL, "densities must be positive");
  if (!(p->mobility >= 0.0)) return fail(LBM_EINVAL, "mobility must be non-negative");
  if (p->storage < LBM_FP32 || p->storage > LBM_BF16_DEV) return fail(LBM_EINVAL, "unknown storage");
  if (p->body_force != LBM_FB_RHO_G && p->body_force != LBM_FB_RHO_MINUS_RHOL_G)
    return fail(LBM_EINVAL, "unknown body force");
  if (p->variant_flags & ~(LBM_VF_CLAMP_PHI | LBM_VF_BGK)) return fail(LBM_EINVAL, "unknown variant flag");
  const int ndim = p->lattice == LBM_D2Q9 ? 2 : 3;
  const int ax = axis_of(p->lattice);
  for (int d = 0; d < 3; ++d) {
    const int lo = p->bc[2 * d], hi = p->bc[2 * d + 1];
    if (lo < 0 || lo > 4 || hi < 0 || hi > 4) return fail(LBM_EINVAL, "unknown boundary type");
    if (d >= ndim) {
      if (lo != LBM_BC_PERIODIC || hi != LBM_BC_PERIODIC)
        return fail(LBM_EINVAL, "faces of the z axis must be periodic in 2D");
      continue;
    }
    if ((lo == LBM_BC_PERIODIC) != (hi == LBM_BC_PERIODIC)) return fail(LBM_EINVAL, "periodic faces must be paired");
    if (lo == LBM_BC_CONVECTIVE_OUTLET || hi == LBM_BC_VELOCITY_INLET)
      return fail(LBM_EUNSUPPORTED, "inlet only on the minus face, outlet only on the plus face");
    if ((lo == LBM_BC_VELOCITY_INLET || hi == LBM_BC_CONVECTIVE_OUTLET) && d != ax)
      return fail(LBM_EUNSUPPORTED, "inlet/outlet only on the last axis (z in 3D, y in 2D)");
  }
  if (has_bc(*p, LBM_BC_CONVECTIVE_OUTLET)) {
    const int n = ax == 2 ? p->nz : p->ny;
    if (n < 3) return fail(LBM_EINVAL, "outlet axis needs at least 3 nodes");
    if (p->outlet_mode != LBM_OUTLET_LOCAL && p->outlet_mode != LBM_OUTLET_MAX &&
        p->outlet_mode != LBM_OUTLET_AVERAGE)
      return fail(LBM_EINVAL, "unknown convective velocity option");
  }
  return LBM_OK;
}

Layout layout_of(const lbm_params& p) {
  const size_t Q = (size_t)p.lattice;
  const size_t N = (size_t)p.nx * p.ny * p.nz;
  const size_t ps = (size_t)pop_size(p.storage);
  Layout L;
  size_t off = 0;
  L.h = off;
  off = align256(off + Q * N * ps);
  L.g = off;
  off = align256(off + Q * N * ps);
  L.u = off;
  off = align256(off + 3 * N * 4);
  L.phi0 = off;
  off = align256(off + N * 4);
  L.phi1 = off;
  if (p.storage != LBM_FP32) off = align256(off + N * 4);
  L.obuf = off;
  if (has_bc(p, LBM_BC_CONVECTIVE_OUTLET)) off = align256(off + 2 * Q * (size_t)plane_of(p) * 4);
  L.total = off;
  return L;
}

KParams kparams_of(const lbm_params& p) {
  KParams K;
  memset(&K, 0, sizeof K);
  K.nx = p.nx;
  K.ny = p.ny;
  K.nz = p.nz;
  K.N = p.nx * p.ny * p.nz;
  K.plane = plane_of(p);
  K.rho_l = (float)p.rho_l;
  K.drho = (float)(p.rho_h - p.rho_l);
  K.tau_l = (float)p.tau_l;
  K.dtau = (float)(p.tau_h - p.tau_l);
  const double beta = 12.0 * p.sigma / p.xi, kappa = 1.5 * p.sigma * p.xi;  // Eq. beta_kappa_relation
  K.beta4 = (float)(4.0 * beta);
  K.kappa = (float)kappa;
  K.inv_xi = (float)(1.0 / p.xi);
  K.omega_h = (float)(1.0 / (3.0 * p.mobility + 0.5));  // tau_phi = M / cs^2
  K.gx = (float)p.gravity[0];
  K.gy = (float)p.gravity[1];
  K.gz = (float)p.gravity[2];
  K.fb_rhol = p.body_force == LBM_FB_RHO_MINUS_RHOL_G ? (float)p.rho_l : 0.0f;
  for (int f = 0; f < 6; ++f) K.bc[f] = p.bc[f];
  K.in_c0 = (float)p.inlet_center[0];
  K.in_c1 = (float)p.inlet_center[1];
  K.in_R = (float)p.inlet_radius;
  K.in_u = (float)p.inlet_u;
  K.two_over_xi = (float)(2.0 / p.xi);
  K.clamp = (p.variant_flags & LBM_VF_CLAMP_PHI) ? 1 : 0;
  K.has_inlet = has_bc(p, LBM_BC_VELOCITY_INLET) ? 1 : 0;
  K.has_outlet = has_bc(p, LBM_BC_CONVECTIVE_OUTLET) ? 1 : 0;
  K.outlet_mode = p.outlet_mode;
  for (int side = 0; side < 2; ++side) {  // x faces (never inlet or outlet)
    const int b = p.bc[side];
    if (b == LBM_BC_NOSLIP || b == LBM_BC_FREESLIP) K.wbits |= 1 << side;
    if (b == LBM_BC_NOSLIP) K.nsbits |= 1 << side;
  }
  return K;
}

Tiling tiling_of(int nx, int ny, int nz, int bx, int by) {
  Tiling T;
  T.bx = bx;
  T.by = by;
  T.ntx = (nx + bx - 1) / bx;
  T.nty = (ny + by - 1) / by;
  T.ntiles = (nx > 0 && ny > 0) ? T.ntx * T.nty * nz : 0;
  return T;
}

bool axis_periodic(const lbm_params& p, int d) {
  const int ndim = p.lattice == LBM_D2Q9 ? 2 : 3;
  return d >= ndim || p.bc[2 * d] == LBM_BC_PERIODIC;
}

// tiled box (fast path: everything but the face layers of non-periodic y
// and z axes; x walls are wall lanes) and those face layers (general path)
void split_domain(const lbm_params& p, Box& X, Faces& F) {
  const int n[3] = {p.nx, p.ny, p.nz};
  int o[3], e[3];
  for (int d = 0; d < 3; ++d) {
    const bool cut = d > 0 && !axis_periodic(p, d);
    o[d] = cut ? 1 : 0;
    e[d] = cut ? std::max(0, n[d] - 2) : n[d];
  }
  X.x0 = o[0];
  X.y0 = o[1];
  X.z0 = o[2];
  X.nx = e[0];
  X.ny = e[1];
  X.nz = e[2];
  const bool d3 = p.lattice == LBM_D3Q19;
  F.z0 = o[2];
  F.nzb = e[2];
  F.n1 = (d3 && !axis_periodic(p, 1)) ? 2 * p.nx * e[2] : 0;
  const int last = d3 ? 2 : 1;
  F.n2 = axis_periodic(p, last) ? 0 : 2 * plane_of(p);
}

void default_tile(const lbm_params& p, int& bx, int& by) {
  if (p.nx >= 64 && p.nx % 64 == 0) {
    bx = 64;
    by = 4;
  } else {
    bx = 32;
    by = 8;
  }
}

bool tile_ok(int bx, int by) {
  const int t = bx * by;
  return bx >= 16 && bx % 16 == 0 && by >= 1 && t % 64 == 0 && t <= 512;
}

// device table and launch geometry of a set of domains
struct LaunchSet {
  DomDev* d_dom = nullptr;
  float* d_uplane = nullptr;  // convective velocity per domain (plane options)
  bool plane_speed = false;   // some domain takes a plane option
  int* d_task = nullptr;      // z-marching task -> domain (null for a single domain)
  int ntasks = 0, zc = 0;     // z-marching tasks (D3Q19), planes per task (0: tiled kernel)
  int mgrid = 1, mchunk = 1;  // persistent launch of the marching kernel
  int* d_tile = nullptr;  // tile -> domain (null for a single domain)
  int ndom = 0, ntiles = 0, nface = 0, nplane = 0;
  int bx = 64, by = 4, bpc = 4, nt = 0;
  bool wall = false;  // some domain has lateral wall faces (wall lanes in the tiles)
  bool bgk = false;   // BGK operator for the hydrodynamic set (the same for every domain)
  int grid = 1, chunk = 1;
  int pgrid = 1;  // phase-field pass: one block per tile
};

void free_launch(LaunchSet& ls) {
  if (ls.d_dom) (void)hipFree(ls.d_dom);
  if (ls.d_tile) (void)hipFree(ls.d_tile);
  if (ls.d_uplane) (void)hipFree(ls.d_uplane);
  ls.d_uplane = nullptr;
  if (ls.d_task) (void)hipFree(ls.d_task);
  ls.d_task = nullptr;
  ls.d_dom = nullptr;
  ls.d_tile = nullptr;
}

}  // namespace

struct lbm_sim {
  lbm_params P;
  KParams K;
  Tiling T;  // whole-domain tiling of the auxiliary kernels
  Box box;
  Faces faces;
  Layout L;
  int Q, ST;
  size_t N;
  char* base;
  hipStream_t stream;   // caller's stream (all launches)
  hipStream_t cap;      // private stream used only to capture graphs
  long long steps;
  double* part;         // reduction partials (library scratch)
  double* res;          // 2 doubles on the device
  double* res_host;     // pinned
  int ppd;              // reduction partials of the domain
  LaunchSet ls;
  hipGraphExec_t g_pair, g_many;
  int many_pairs;
  float* phi(int i) { return (float*)(base + (i == 0 ? L.phi0 : L.phi1)); }
  void* h() { return base + L.h; }
  void* g() { return base + L.g; }
  float* u() { return (float*)(base + L.u); }
  float* obuf() { return K.has_outlet ? (float*)(base + L.obuf) : nullptr; }
  int parity() const { return (int)(steps & 1); }
  // 16-bit forms ping-pong two phase-field buffers: at parity p the stored
  // populations were encoded with phi[p] and this step's phi goes to phi[1-p].
  float* ref_buf(int par) { return ST == LBM_FP32 ? phi(0) : phi(par); }
  float* out_buf(int par) { return ST == LBM_FP32 ? phi(0) : phi(1 - par); }
  KBufs bufs(int par) {
    KBufs B;
    B.h = h();
    B.g = g();
    B.u = u();
    B.phi = out_buf(par);
    B.phi_out = out_buf(par);
    B.ref = ref_buf(par);
    B.obuf = obuf();
    return B;
  }
};

namespace {

// Fill the device table of the domains `v[0..n)` with launch shape (bx, by,
// blocks per CU, store hint); allocates the table (replacing any old one).
int build_launch(LaunchSet& ls, lbm_sim* const* v, int n, int bx, int by, int bpc, int nt) {
  std::vector<DomDev> dom(n);
  std::vector<int> tile_dom, task_dom;
  int tb = 0, fb = 0, pb = 0, kb = 0;
  const int zc = ls.zc;
  bool wall = false;
  const bool bgk = (v[0]->P.variant_flags & LBM_VF_BGK) != 0;
  for (int d = 0; d < n; ++d) {
    if (((v[d]->P.variant_flags & LBM_VF_BGK) != 0) != bgk)
      return fail(LBM_EINVAL, "all domains of a batch must use the same collision operator");
    lbm_sim* s = v[d];
    DomDev& m = dom[d];
    memset(&m, 0, sizeof m);
    m.K = s->K;
    for (int par = 0; par < 2; ++par) {
      m.B[par] = s->bufs(par);
      m.Bo[par] = s->bufs(par);
      m.Bo[par].ref = s->out_buf(par);  // the outlet decodes what this step wrote
    }
    m.X = s->box;
    m.F = s->faces;
    const Tiling TB = tiling_of(s->box.nx, s->box.ny, s->box.nz, bx, by);
    m.ntx = TB.ntx;
    m.nty = TB.nty;
    m.ntiles = TB.ntiles;
    m.tile_base = tb;
    m.face_base = fb;
    m.plane_base = pb;
    if (n > 1) tile_dom.insert(tile_dom.end(), (size_t)TB.ntiles, d);
    tb += TB.ntiles;
    m.task_base = kb;
    // zc = 0 selects the tiled kernel: no marching tasks
    const int ntask = (zc > 0 && s->box.nz > 0) ? TB.ntx * TB.nty * ((s->box.nz + zc - 1) / zc) : 0;
    if (n > 1) task_dom.insert(task_dom.end(), (size_t)ntask, d);
    kb += ntask;
    fb += s->faces.n1 + s->faces.n2;
    wall |= s->K.wbits != 0;
    pb += s->K.has_outlet ? s->K.plane : 0;
  }
  free_launch(ls);
  HIPCHK(hipMalloc(&ls.d_uplane, sizeof(float) * n));
  HIPCHK(hipMemset(ls.d_uplane, 0, sizeof(float) * n));
  ls.plane_speed = false;
  for (int d = 0; d < n; ++d) {
    dom[d].uplane = ls.d_uplane + d;
    ls.plane_speed |= dom[d].K.has_outlet && dom[d].K.outlet_mode != 0;
  }
  ls.wall = wall;
  ls.bgk = bgk;
  ls.ndom = n;
  ls.ntiles = tb;
  ls.ntasks = kb;
  ls.nface = fb;
  ls.nplane = pb;
  ls.bx = bx;
  ls.by = by;
  ls.bpc = bpc;
  ls.nt = nt;
  HIPCHK(hipMalloc(&ls.d_dom, sizeof(DomDev) * n));
  HIPCHK(hipMemcpy(ls.d_dom, dom.data(), sizeof(DomDev) * n, hipMemcpyHostToDevice));
  if (n > 1 && kb) {
    HIPCHK(hipMalloc(&ls.d_task, sizeof(int) * kb));
    HIPCHK(hipMemcpy(ls.d_task, task_dom.data(), sizeof(int) * kb, hipMemcpyHostToDevice));
  }
  if (n > 1 && tb) {
    HIPCHK(hipMalloc(&ls.d_tile, sizeof(int) * tb));
    HIPCHK(hipMemcpy(ls.d_tile, tile_dom.data(), sizeof(int) * tb, hipMemcpyHostToDevice));
  }
  int dev = 0, cus = 256;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // persistent launch: about bpc resident blocks per compute unit, each
  // walking a contiguous chunk of tiles; bpc = 0: one block per tile (the
  // dispatcher refills the compute units as blocks end)
  const int want = bpc > 0 ? std::max(1, std::min(std::max(tb, 1), cus * bpc)) : std::max(tb, 1);
  ls.chunk = std::max(1, (tb + want - 1) / want);
  ls.grid = std::max(1, (tb + ls.chunk - 1) / ls.chunk);
  // the phase-field pass (one read per population, one write) runs fastest
  // as one block per tile in every measured case, whatever suits the step
  ls.pgrid = std::max(tb, 1);
  const int mwant = bpc > 0 ? std::max(1, std::min(std::max(kb, 1), cus * bpc)) : std::max(kb, 1);
  ls.mchunk = std::max(1, (kb + mwant - 1) / mwant);
  ls.mgrid = std::max(1, (kb + ls.mchunk - 1) / ls.mchunk);
  return LBM_OK;
}

template <int Q, int ST, int PAR>
void launch_phi_set(const LaunchSet& ls, hipStream_t st) {
  const dim3 gi(ls.pgrid), bi(ls.bx * ls.by);
  if (ls.ntiles && ls.wall)
    hipLaunchKernelGGL((kb_interior<Q, ST, PAR, false, true, true, false>), gi, bi, 0, st, ls.d_dom, ls.d_tile,
                       ls.ntiles, 1, ls.bx, ls.by);
  else if (ls.ntiles)
    hipLaunchKernelGGL((kb_interior<Q, ST, PAR, false, true, false, false>), gi, bi, 0, st, ls.d_dom,
                       ls.d_tile, ls.ntiles, 1, ls.bx, ls.by);
  if (ls.nface)
    hipLaunchKernelGGL((kb_faces<Q, ST, PAR, false, true, false>), dim3((ls.nface + 255) / 256), dim3(256), 0,
                       st, ls.d_dom, ls.ndom, ls.nface);
}

template <int Q, int ST, int PAR, bool NT, bool BGK>
void launch_collide_op(const LaunchSet& ls, hipStream_t st) {
  const dim3 gi(ls.grid), bi(ls.bx * ls.by);
  if (Q == 19 && ls.zc > 0) {  // z-marching interior with the LDS phase-field ring
    const dim3 gm(ls.mgrid);
    const size_t lds = sizeof(float) * 5 * (size_t)(ls.bx + 2) * (ls.by + 2);
    if (ls.ntasks && ls.wall)
      hipLaunchKernelGGL((kb_march<ST, PAR, NT, true, BGK>), gm, bi, lds, st, ls.d_dom, ls.d_task, ls.ntasks,
                         ls.mchunk, ls.bx, ls.by, ls.zc);
    else if (ls.ntasks)
      hipLaunchKernelGGL((kb_march<ST, PAR, NT, false, BGK>), gm, bi, lds, st, ls.d_dom, ls.d_task, ls.ntasks,
                         ls.mchunk, ls.bx, ls.by, ls.zc);
  } else if (ls.ntiles && ls.wall)
    hipLaunchKernelGGL((kb_interior<Q, ST, PAR, NT, false, true, BGK>), gi, bi, 0, st, ls.d_dom, ls.d_tile,
                       ls.ntiles, ls.chunk, ls.bx, ls.by);
  else if (ls.ntiles)
    hipLaunchKernelGGL((kb_interior<Q, ST, PAR, NT, false, false, BGK>), gi, bi, 0, st, ls.d_dom, ls.d_tile,
                       ls.ntiles, ls.chunk, ls.bx, ls.by);
  if (ls.nface)
    hipLaunchKernelGGL((kb_faces<Q, ST, PAR, NT, false, BGK>), dim3((ls.nface + 255) / 256), dim3(256), 0, st,
                       ls.d_dom, ls.ndom, ls.nface);
}

template <int Q, int ST, int PAR, bool NT>
void launch_collide_set(const LaunchSet& ls, hipStream_t st) {
  if (ls.bgk)
    launch_collide_op<Q, ST, PAR, NT, true>(ls, st);
  else
    launch_collide_op<Q, ST, PAR, NT, false>(ls, st);
}

// one step of parity `par`: phase-field pass, fused step, outlet planes;
// events (nullable) bracket the three phases
template <int Q, int ST>
hipError_t launch_step_t(const LaunchSet& ls, int par, hipStream_t st, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], st);
  if (par == 0)
    launch_phi_set<Q, ST, 0>(ls, st);
  else
    launch_phi_set<Q, ST, 1>(ls, st);
  if (ev) (void)hipEventRecord(ev[1], st);
  if (par == 0) {
    if (ls.nt)
      launch_collide_set<Q, ST, 0, true>(ls, st);
    else
      launch_collide_set<Q, ST, 0, false>(ls, st);
  } else {
    if (ls.nt)
      launch_collide_set<Q, ST, 1, true>(ls, st);
    else
      launch_collide_set<Q, ST, 1, false>(ls, st);
  }
  if (ev) (void)hipEventRecord(ev[2], st);
  if (ls.nplane) {
    const dim3 gp((ls.nplane + 255) / 256), bp(256);
    if (ls.plane_speed) hipLaunchKernelGGL((k_outlet_speed<Q>), dim3(ls.ndom), bp, 0, st, ls.d_dom);
    if (par == 0)
      hipLaunchKernelGGL((kb_outlet<Q, ST, 0>), gp, bp, 0, st, ls.d_dom, ls.ndom, ls.nplane);
    else
      hipLaunchKernelGGL((kb_outlet<Q, ST, 1>), gp, bp, 0, st, ls.d_dom, ls.ndom, ls.nplane);
  }
  if (ev) (void)hipEventRecord(ev[3], st);
  return hipGetLastError();
}

hipError_t launch_step(const LaunchSet& ls, int Q, int ST, int par, hipStream_t st, hipEvent_t* ev = nullptr) {
  if (Q == 9) {
    if (ST == 0) return launch_step_t<9, 0>(ls, par, st, ev);
    if (ST == 1) return launch_step_t<9, 1>(ls, par, st, ev);
    return launch_step_t<9, 2>(ls, par, st, ev);
  }
  if (ST == 0) return launch_step_t<19, 0>(ls, par, st, ev);
  if (ST == 1) return launch_step_t<19, 1>(ls, par, st, ev);
  return launch_step_t<19, 2>(ls, par, st, ev);
}

template <int Q, int ST>
hipError_t launch_phi_t(const LaunchSet& ls, int par, hipStream_t st) {
  if (par == 0)
    launch_phi_set<Q, ST, 0>(ls, st);
  else
    launch_phi_set<Q, ST, 1>(ls, st);
  return hipGetLastError();
}


// ---- FP64 reductions over a domain table -------------------------------------
// Partial sums per domain: one per 64 Ki nodes of the largest domain, at
// least 1 and at most 1024, and at most kReduceMaxParts over all domains
// (the capacity of the allocation-free reduction's scratch array).  Both
// batch reductions use this count, so they give bitwise the same sums.

int reduce_ppd(size_t max_nodes, int ndom) {
  size_t p = (max_nodes + 65535) / 65536;
  p = std::min<size_t>(std::max<size_t>(p, 1), 1024);
  p = std::min<size_t>(p, std::max<size_t>(1, (size_t)kReduceMaxParts / (size_t)std::max(ndom, 1)));
  return (int)p;
}

hipError_t launch_phi_ls(const LaunchSet& ls, int Q, int ST, int par, hipStream_t st) {
  if (Q == 9) {
    if (ST == 0) return launch_phi_t<9, 0>(ls, par, st);
    if (ST == 1) return launch_phi_t<9, 1>(ls, par, st);
    return launch_phi_t<9, 2>(ls, par, st);
  }
  if (ST == 0) return launch_phi_t<19, 0>(ls, par, st);
  if (ST == 1) return launch_phi_t<19, 1>(ls, par, st);
  return launch_phi_t<19, 2>(ls, par, st);
}

// phase-field pass of every domain of the set, then per-domain sums of phi and
// kinetic energy: part holds ndom * ppd pairs, out receives 2 * ndom doubles
hipError_t launch_reduce(const LaunchSet& ls, int Q, int ST, int par, int ppd, double* part, double* out,
                         hipStream_t st) {
  hipError_t e = launch_phi_ls(ls, Q, ST, par, st);
  if (e != hipSuccess) return e;
  const dim3 gp((unsigned)(ls.ndom * ppd)), bp(256);
  if (par == 0)
    hipLaunchKernelGGL(k_reduce_partial<0>, gp, bp, 0, st, (const DomDev*)ls.d_dom, ppd, part);
  else
    hipLaunchKernelGGL(k_reduce_partial<1>, gp, bp, 0, st, (const DomDev*)ls.d_dom, ppd, part);
  hipLaunchKernelGGL(k_reduce_final, dim3(ls.ndom), bp, 0, st, (const double*)part, ppd, out);
  return hipGetLastError();
}

hipError_t launch_phi(lbm_sim* s) { return launch_phi_ls(s->ls, s->Q, s->ST, s->parity(), s->stream); }

// ---- auxiliary kernels of one domain ----------------------------------------
template <int Q, int ST>
hipError_t launch_init_t(lbm_sim* s, const float* phi0, const float* u0) {
  const dim3 grid(s->T.ntiles), block(s->T.bx * s->T.by);
  KBufs B = s->bufs(0);
  hipLaunchKernelGGL((k_init<Q, ST>), grid, block, 0, s->stream, s->K, B, phi0, u0, s->T);
  return hipGetLastError();
}

template <int Q, int ST>
hipError_t launch_export_t(lbm_sim* s, float* ho, float* go, float* uo) {
  const int par = s->parity();
  const dim3 grid(s->T.ntiles), block(s->T.bx * s->T.by);
  KBufs B = s->bufs(par);
  if (par == 0)
    hipLaunchKernelGGL((k_export<Q, ST, 0>), grid, block, 0, s->stream, s->K, B, ho, go, uo, s->T);
  else
    hipLaunchKernelGGL((k_export<Q, ST, 1>), grid, block, 0, s->stream, s->K, B, ho, go, uo, s->T);
  return hipGetLastError();
}

template <int Q, int ST>
hipError_t launch_import_t(lbm_sim* s, const float* hi, const float* gi, const float* ui) {
  const dim3 grid(s->T.ntiles), block(s->T.bx * s->T.by);
  KBufs B = s->bufs(0);
  hipLaunchKernelGGL((k_import_ref<Q>), grid, block, 0, s->stream, s->K, hi, s->ref_buf(0), s->T);
  hipLaunchKernelGGL((k_import<Q, ST>), grid, block, 0, s->stream, s->K, B, hi, gi, ui, s->T);
  return hipGetLastError();
}

template <int Q, int ST>
hipError_t launch_pressure_t(lbm_sim* s, float* po) {
  const int par = s->parity();
  const dim3 grid(s->T.ntiles), block(s->T.bx * s->T.by);
  KBufs B = s->bufs(par);
  if (par == 0)
    hipLaunchKernelGGL((k_pressure<Q, ST, 0>), grid, block, 0, s->stream, s->K, B, po, s->T);
  else
    hipLaunchKernelGGL((k_pressure<Q, ST, 1>), grid, block, 0, s->stream, s->K, B, po, s->T);
  return hipGetLastError();
}

#define DISPATCH(fn, s, ...)                                                          \
  ((s)->Q == 9 ? ((s)->ST == 0   ? fn<9, 0>((s), __VA_ARGS__)                          \
                  : (s)->ST == 1 ? fn<9, 1>((s), __VA_ARGS__)                          \
                                 : fn<9, 2>((s), __VA_ARGS__))                         \
               : ((s)->ST == 0   ? fn<19, 0>((s), __VA_ARGS__)                         \
                  : (s)->ST == 1 ? fn<19, 1>((s), __VA_ARGS__)                         \
                                 : fn<19, 2>((s), __VA_ARGS__)))

// ---- graphs ------------------------------------------------------------------
void drop_graph(hipGraphExec_t& g) {
  if (g) (void)hipGraphExecDestroy(g);
  g = nullptr;
}

int capture_pairs(const LaunchSet& ls, int Q, int ST, hipStream_t cap, int pairs, hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  for (int i = 0; i < pairs && err == hipSuccess; ++i) {
    err = launch_step(ls, Q, ST, 0, cap);
    if (err == hipSuccess) err = launch_step(ls, Q, ST, 1, cap);
  }
  hipError_t e2 = hipStreamEndCapture(cap, &graph);
  if (err != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(LBM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(err != hipSuccess ? err : e2));
  }
  hipError_t e3 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e3 != hipSuccess) return fail(LBM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e3));
  return LBM_OK;
}

void drop_graphs(lbm_sim* s) {
  drop_graph(s->g_pair);
  drop_graph(s->g_many);
}

int build_graphs(lbm_sim* s) {
  drop_graphs(s);
  // about 4M node updates or more per graph launch
  s->many_pairs = (int)std::max<size_t>(1, std::min<size_t>(64, (size_t)4000000 / std::max<size_t>(1, s->N)));
  int rc = capture_pairs(s->ls, s->Q, s->ST, s->cap, 1, &s->g_pair);
  if (rc) return rc;
  if (s->many_pairs > 1) rc = capture_pairs(s->ls, s->Q, s->ST, s->cap, s->many_pairs, &s->g_many);
  return rc;
}

// new launch shape; with `graphs` the step graphs are captured again here, so
// that lbm_step only replays them
int set_launch(lbm_sim* s, int bx, int by, int bpc, int nt, bool graphs) {
  drop_graphs(s);
  lbm_sim* v[1] = {s};
  int rc = build_launch(s->ls, v, 1, bx, by, bpc, nt);
  if (rc == LBM_OK && graphs) rc = build_graphs(s);
  return rc;
}

// simulation object on an existing state buffer; no launch.  `graphs`: capture
// the step graphs now (a batch's per-domain views step through the batch's)
lbm_sim* new_sim(const lbm_params* p, char* base, hipStream_t stream, int* rc, bool graphs) {
  lbm_sim* s = new lbm_sim();
  s->P = *p;
  s->K = kparams_of(*p);
  s->L = layout_of(*p);
  s->Q = p->lattice;
  s->ST = p->storage;
  s->N = (size_t)p->nx * p->ny * p->nz;
  s->base = base;
  s->stream = stream;
  s->steps = 0;
  s->g_pair = s->g_many = nullptr;
  s->many_pairs = 1;
  s->part = s->res = s->res_host = nullptr;
  s->cap = nullptr;
  int bx, by;
  default_tile(*p, bx, by);
  split_domain(*p, s->box, s->faces);
  s->T = tiling_of(p->nx, p->ny, p->nz, bx, by);
  s->ppd = reduce_ppd(s->N, 1);
  hipError_t e = hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&s->part, sizeof(double) * 2 * s->ppd);
  if (e == hipSuccess) e = hipMalloc(&s->res, sizeof(double) * 2);
  if (e == hipSuccess) e = hipHostMalloc(&s->res_host, sizeof(double) * 2, hipHostMallocDefault);
  if (e != hipSuccess) {
    *rc = fail(LBM_ENOMEM, std::string("library scratch: ") + hipGetErrorString(e));
    lbm_destroy(s);
    return nullptr;
  }
  *rc = set_launch(s, bx, by, 4, 0, graphs);
  if (*rc) {
    lbm_destroy(s);
    return nullptr;
  }
  return s;
}

// initial populations (even-parity slots) from phi0, u0
int init_kernels(lbm_sim* s, const float* phi0_dev, const float* u0_dev) {
  hipError_t e = DISPATCH(launch_init_t, s, phi0_dev, u0_dev);
  if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("init kernel: ") + hipGetErrorString(e));
  // the 16-bit forms decode with the reader's phase field: phi0
  if (s->ST != LBM_FP32) {
    e = hipMemcpyAsync(s->ref_buf(0), phi0_dev, s->N * sizeof(float), hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("init copy: ") + hipGetErrorString(e));
  }
  return LBM_OK;
}

// mean ms per eager step over n steps (events around the whole step)
int time_steps(const LaunchSet& ls, int Q, int ST, hipStream_t st, long long& steps, int n, double* ms) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t err = hipEventRecord(e0, st);
  for (int i = 0; i < n && err == hipSuccess; ++i) {
    err = launch_step(ls, Q, ST, (int)(steps & 1), st);
    steps += 1;
  }
  if (err == hipSuccess) err = hipEventRecord(e1, st);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(LBM_EDEVICE, hipGetErrorString(err));
  *ms = t / n;
  return LBM_OK;
}

// per-phase mean ms over n eager steps
int phase_times(const LaunchSet& ls, int Q, int ST, hipStream_t st, long long& steps, int n, double* out) {
  hipEvent_t ev[4];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  double acc[3] = {0, 0, 0};
  hipError_t err = hipSuccess;
  for (int i = 0; i < n && err == hipSuccess; ++i) {
    err = launch_step(ls, Q, ST, (int)(steps & 1), st, ev);
    steps += 1;
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    for (int k = 0; k < 3 && err == hipSuccess; ++k) {
      float ms = 0.f;
      err = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      acc[k] += ms;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (err != hipSuccess) return fail(LBM_EDEVICE, hipGetErrorString(err));
  for (int k = 0; k < 3; ++k) out[k] = acc[k] / n;
  return LBM_OK;
}

struct TuneEntry {
  int bx, by, bpc, nt, zc;
  double ms;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune_cache;

const int kTiles[][2] = {{64, 4}, {128, 2}, {256, 1}, {32, 8}, {64, 8}, {128, 4}, {32, 4}, {16, 16}};
const int kBpc[] = {0, 2, 4, 8};
// planes per z-marching task tried by the autotuners (D3Q19; 0 = tiled kernel)
const int kZc[] = {0, 32};

// Candidate tiles of the autotuner for boxes whose rows are `w` nodes wide
// (0: widths differ): the fixed list without mostly idle shapes, plus
// whole-row tiles (every wave then covers contiguous nodes).
std::vector<std::pair<int, int>> tile_candidates(int w, int ny) {
  std::vector<std::pair<int, int>> out;
  for (const auto& cb : kTiles) {
    if (w > 0 && cb[0] > 16 && cb[0] >= 2 * w) continue;
    if (cb[1] > 1 && cb[1] > ny) continue;
    out.emplace_back(cb[0], cb[1]);
  }
  if (w > 0 && w % 16 == 0)
    for (int by = 1; by <= 8; by *= 2)
      if (tile_ok(w, by) && by <= ny &&
          std::find(out.begin(), out.end(), std::make_pair(w, by)) == out.end())
        out.emplace_back(w, by);
  return out;
}

std::string params_key(const lbm_params& p) {
  char buf[200];
  snprintf(buf, sizeof buf, "q%d st%d %dx%dx%d bc%d%d%d%d%d%d", p.lattice, p.storage, p.nx, p.ny, p.nz, p.bc[0],
           p.bc[1], p.bc[2], p.bc[3], p.bc[4], p.bc[5]);
  return buf;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }
const char* lbm_version(void) { return "lbm-pf-gfx950 0.2"; }

int lbm_state_bytes(const lbm_params* p, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "null output");
  *bytes = layout_of(*p).total;
  return LBM_OK;
}

int lbm_init(const lbm_params* p, const float* phi0_dev, const float* u0_dev, void* state_dev,
             size_t state_bytes, void* stream, lbm_sim** out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out || !phi0_dev || !state_dev) return fail(LBM_EINVAL, "null pointer argument");
  const Layout L = layout_of(*p);
  if (state_bytes < L.total) return fail(LBM_ENOMEM, "state buffer smaller than lbm_state_bytes()");
  if (((uintptr_t)state_dev) & 255) return fail(LBM_EINVAL, "state buffer must be 256-byte aligned");
  lbm_sim* s = new_sim(p, (char*)state_dev, (hipStream_t)stream, &rc, true);
  if (!s) return rc;
  rc = init_kernels(s, phi0_dev, u0_dev);
  if (rc) {
    lbm_destroy(s);
    return rc;
  }
  *out = s;
  return LBM_OK;
}

int lbm_step(lbm_sim* s, int n) {
  if (!s || n < 0) return fail(LBM_EINVAL, "bad handle or step count");
  if (n >= 2 && !s->g_pair) return fail(LBM_EINVAL, "no step graph (an autotune trial left the launch without one)");
  while (n > 0) {
    if (s->parity() == 1 || n == 1) {
      HIPCHK(launch_step(s->ls, s->Q, s->ST, s->parity(), s->stream));
      s->steps += 1;
      n -= 1;
    } else if (s->g_many && n >= 2 * s->many_pairs) {
      HIPCHK(hipGraphLaunch(s->g_many, s->stream));
      s->steps += 2 * s->many_pairs;
      n -= 2 * s->many_pairs;
    } else {
      HIPCHK(hipGraphLaunch(s->g_pair, s->stream));
      s->steps += 2;
      n -= 2;
    }
  }
  return LBM_OK;
}

long long lbm_steps_done(const lbm_sim* s) { return s ? s->steps : -1; }

int lbm_fields(lbm_sim* s, unsigned mask, float* phi_dev, float* u_dev, float* p_dev) {
  if (!s) return fail(LBM_EINVAL, "null handle");
  if ((mask & LBM_FIELD_PHI) && !phi_dev) return fail(LBM_EINVAL, "null phi buffer");
  if ((mask & LBM_FIELD_U) && !u_dev) return fail(LBM_EINVAL, "null u buffer");
  if ((mask & LBM_FIELD_P) && !p_dev) return fail(LBM_EINVAL, "null p buffer");
  if (mask & LBM_FIELD_PHI) {
    HIPCHK(launch_phi(s));
    HIPCHK(hipMemcpyAsync(phi_dev, s->out_buf(s->parity()), s->N * sizeof(float), hipMemcpyDeviceToDevice,
                          s->stream));
  }
  if (mask & LBM_FIELD_U)
    HIPCHK(hipMemcpyAsync(u_dev, s->u(), 3 * s->N * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  if (mask & LBM_FIELD_P) HIPCHK(DISPATCH(launch_pressure_t, s, p_dev));
  return LBM_OK;
}

int lbm_reduce(lbm_sim* s, double* mass, double* kinetic) {
  if (!s || !mass || !kinetic) return fail(LBM_EINVAL, "null argument");
  HIPCHK(launch_reduce(s->ls, s->Q, s->ST, s->parity(), s->ppd, s->part, s->res, s->stream));
  HIPCHK(hipMemcpyAsync(s->res_host, s->res, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  *mass = s->res_host[0];
  *kinetic = s->res_host[1];
  if (!std::isfinite(*mass) || !std::isfinite(*kinetic))
    return fail(LBM_EUNSTABLE, "non-finite mass or kinetic energy");
  return LBM_OK;
}

int lbm_export_state(lbm_sim* s, float* h_dev, float* g_dev, float* u_dev) {
  if (!s) return fail(LBM_EINVAL, "null handle");
  HIPCHK(DISPATCH(launch_export_t, s, h_dev, g_dev, u_dev));
  return LBM_OK;
}

int lbm_import_state(lbm_sim* s, const float* h_dev, const float* g_dev, const float* u_dev) {
  if (!s || !h_dev || !g_dev || !u_dev) return fail(LBM_EINVAL, "null argument");
  s->steps = 0;  // canonical state is stored in even-parity slots
  HIPCHK(DISPATCH(launch_import_t, s, h_dev, g_dev, u_dev));
  return LBM_OK;
}

int lbm_checkpoint_bytes(const lbm_sim* s, size_t* bytes) {
  if (!s || !bytes) return fail(LBM_EINVAL, "null argument");
  *bytes = s->L.total + 64;
  return LBM_OK;
}

int lbm_save(lbm_sim* s, void* host_buf, size_t bytes) {
  if (!s || !host_buf || bytes < s->L.total + 64) return fail(LBM_EINVAL, "bad checkpoint buffer");
  char* hb = (char*)host_buf;
  memset(hb, 0, 64);
  memcpy(hb, "LBMPF001", 8);
  memcpy(hb + 8, &s->steps, sizeof(long long));
  memcpy(hb + 16, &s->L.total, sizeof(size_t));
  HIPCHK(hipStreamSynchronize(s->stream));
  HIPCHK(hipMemcpy(hb + 64, s->base, s->L.total, hipMemcpyDeviceToHost));
  return LBM_OK;
}

int lbm_load(lbm_sim* s, const void* host_buf, size_t bytes) {
  if (!s || !host_buf || bytes < s->L.total + 64) return fail(LBM_EINVAL, "bad checkpoint buffer");
  const char* hb = (const char*)host_buf;
  size_t tot = 0;
  memcpy(&tot, hb + 16, sizeof(size_t));
  if (memcmp(hb, "LBMPF001", 8) != 0 || tot != s->L.total)
    return fail(LBM_EINVAL, "checkpoint does not match this simulation");
  HIPCHK(hipStreamSynchronize(s->stream));
  HIPCHK(hipMemcpy(s->base, hb + 64, s->L.total, hipMemcpyHostToDevice));
  memcpy(&s->steps, hb + 8, sizeof(long long));
  return LBM_OK;
}

int lbm_set_tile(lbm_sim* s, int bx, int by) {
  if (!s) return fail(LBM_EINVAL, "null handle");
  if (!tile_ok(bx, by)) return fail(LBM_EINVAL, "tile must have bx % 16 == 0 and bx*by a multiple of 64 up to 512");
  return set_launch(s, bx, by, s->ls.bpc, s->ls.nt, true);
}

int lbm_set_store_hint(lbm_sim* s, int nontemporal) {
  if (!s) return fail(LBM_EINVAL, "null handle");
  return set_launch(s, s->ls.bx, s->ls.by, s->ls.bpc, nontemporal ? 1 : 0, true);
}

int lbm_set_blocks_per_cu(lbm_sim* s, int blocks_per_cu) {
  if (!s || blocks_per_cu < 0 || blocks_per_cu > 64) return fail(LBM_EINVAL, "bad argument");
  return set_launch(s, s->ls.bx, s->ls.by, blocks_per_cu, s->ls.nt, true);
}

int lbm_set_zchunk(lbm_sim* s, int planes) {
  if (!s || planes < 0 || planes > 4096) return fail(LBM_EINVAL, "bad argument");
  s->ls.zc = planes;
  return set_launch(s, s->ls.bx, s->ls.by, s->ls.bpc, s->ls.nt, true);
}

int lbm_get_zchunk(const lbm_sim* s, int* planes) {
  if (!s || !planes) return fail(LBM_EINVAL, "null argument");
  *planes = s->ls.zc;
  return LBM_OK;
}

int lbm_get_blocks_per_cu(const lbm_sim* s, int* blocks_per_cu) {
  if (!s || !blocks_per_cu) return fail(LBM_EINVAL, "null argument");
  *blocks_per_cu = s->ls.bpc;
  return LBM_OK;
}

int lbm_get_tile(const lbm_sim* s, int* bx, int* by) {
  if (!s || !bx || !by) return fail(LBM_EINVAL, "null argument");
  *bx = s->ls.bx;
  *by = s->ls.by;
  return LBM_OK;
}

int lbm_kernel_times(lbm_sim* s, int n, double* out_ms) {
  if (!s || n < 1 || !out_ms) return fail(LBM_EINVAL, "bad argument");
  return phase_times(s->ls, s->Q, s->ST, s->stream, s->steps, n, out_ms);
}

int lbm_autotune(lbm_sim* s, int trial_steps, int* bx_out, int* by_out, int* nt_out, double* ms_out) {
  if (!s || trial_steps < 1) return fail(LBM_EINVAL, "bad argument");
  const std::string key = params_key(s->P);
  TuneEntry best = {s->ls.bx, s->ls.by, s->ls.bpc, s->ls.nt, s->ls.zc, 1e30};
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      best = it->second;
      cached = true;
    }
  }
  if (!cached) {
    for (const auto& cb : tile_candidates(std::max(1, s->box.nx), s->P.ny)) {
      const int bx = cb.first, by = cb.second;
      for (int bp : kBpc)
        for (int nt = 0; nt < 2; ++nt)
          for (int zc : kZc) {
            if (zc && s->Q != 19) continue;
            s->ls.zc = zc;
            int rc = set_launch(s, bx, by, bp, nt, false);
            double ms = 0.0;
            if (rc == LBM_OK) rc = time_steps(s->ls, s->Q, s->ST, s->stream, s->steps, 2, &ms);  // warm-up
            if (rc == LBM_OK) rc = time_steps(s->ls, s->Q, s->ST, s->stream, s->steps, trial_steps, &ms);
            if (rc) return rc;
            if (ms < best.ms) best = {bx, by, bp, nt, zc, ms};
          }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  s->ls.zc = best.zc;
  int rc = set_launch(s, best.bx, best.by, best.bpc, best.nt, true);
  if (rc) return rc;
  if (bx_out) *bx_out = best.bx;
  if (by_out) *by_out = best.by;
  if (nt_out) *nt_out = best.nt;
  if (ms_out) *ms_out = best.ms;
  return LBM_OK;
}

void lbm_destroy(lbm_sim* s) {
  if (!s) return;
  drop_graphs(s);
  free_launch(s->ls);
  if (s->part) (void)hipFree(s->part);
  if (s->res) (void)hipFree(s->res);
  if (s->res_host) (void)hipHostFree(s->res_host);
  if (s->cap) (void)hipStreamDestroy(s->cap);
  delete s;
}

}  // extern "C"

// ===========================================================================
// Batched form: many independent domains advanced by the same launches
// ===========================================================================
struct lbm_batch {
  int ndom = 0, Q = 0, ST = 0;
  std::vector<lbm_sim*> views;  // one per domain, on its slice of the arena
  std::vector<size_t> off;
  char* base = nullptr;
  hipStream_t stream = nullptr, cap = nullptr;
  LaunchSet ls;
  long long steps = 0;
  hipGraphExec_t g_pair = nullptr;
  int* d_count = nullptr;
  int count_cap = 0;
  int ppd = 1;                   // reduction partials per domain
  double* part = nullptr;        // ndom * ppd pairs (library scratch)
  double* res = nullptr;         // 2 * ndom doubles on the device
  double* res_host = nullptr;    // pinned copy of res
  double* scratch = nullptr;     // this device's copy of the static scratch array
};

namespace {

size_t batch_layout(int ndom, const lbm_params* p, std::vector<size_t>& off) {
  off.resize(ndom);
  size_t tot = 0;
  for (int d = 0; d < ndom; ++d) {
    off[d] = tot;
    tot = align256(tot + layout_of(p[d]).total);
  }
  return tot;
}

int batch_validate(int ndom, const lbm_params* p) {
  if (ndom < 1 || !p) return fail(LBM_EINVAL, "need at least one domain");
  for (int d = 0; d < ndom; ++d) {
    int rc = validate(&p[d]);
    if (rc) return fail(rc, "domain " + std::to_string(d) + ": " + g_err);
    if (p[d].lattice != p[0].lattice || p[d].storage != p[0].storage)
      return fail(LBM_EINVAL, "all domains of a batch share lattice and storage");
    if ((p[d].variant_flags ^ p[0].variant_flags) & LBM_VF_BGK)
      return fail(LBM_EINVAL, "all domains of a batch must use the same collision operator");
  }
  return LBM_OK;
}

// new launch shape; with `graphs` the step-pair graph is captured again here
int batch_set_launch(lbm_batch* b, int bx, int by, int bpc, int nt, bool graphs) {
  drop_graph(b->g_pair);
  int rc = build_launch(b->ls, b->views.data(), b->ndom, bx, by, bpc, nt);
  if (rc == LBM_OK && graphs) rc = capture_pairs(b->ls, b->Q, b->ST, b->cap, 1, &b->g_pair);
  return rc;
}

void batch_sync_views(lbm_batch* b) {
  for (auto* v : b->views) v->steps = b->steps;
}

std::string batch_key(const lbm_batch* b) {
  std::string k = "batch n" + std::to_string(b->ndom);
  for (auto* v : b->views) k += " " + params_key(v->P);
  return k;
}

}  // namespace

extern "C" {

int lbm_batch_state_bytes(int ndom, const lbm_params* p, size_t* bytes) {
  int rc = batch_validate(ndom, p);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "null output");
  std::vector<size_t> off;
  *bytes = batch_layout(ndom, p, off);
  return LBM_OK;
}

int lbm_batch_init(int ndom, const lbm_params* p, const float* const* phi0_dev, const float* const* u0_dev,
                   void* state_dev, size_t state_bytes, void* stream, lbm_batch** out) {
  int rc = batch_validate(ndom, p);
  if (rc) return rc;
  if (!out || !phi0_dev || !state_dev) return fail(LBM_EINVAL, "null pointer argument");
  if (((uintptr_t)state_dev) & 255) return fail(LBM_EINVAL, "state buffer must be 256-byte aligned");
  lbm_batch* b = new lbm_batch();
  const size_t total = batch_layout(ndom, p, b->off);
  if (state_bytes < total) {
    delete b;
    return fail(LBM_ENOMEM, "state buffer smaller than lbm_batch_state_bytes()");
  }
  b->ndom = ndom;
  b->Q = p[0].lattice;
  b->ST = p[0].storage;
  b->base = (char*)state_dev;
  b->stream = (hipStream_t)stream;
  b->views.assign(ndom, nullptr);
  for (int d = 0; d < ndom && rc == LBM_OK; ++d) {
    if (!phi0_dev[d]) {
      rc = fail(LBM_EINVAL, "null phi0 for domain " + std::to_string(d));
      break;
    }
    b->views[d] = new_sim(&p[d], b->base + b->off[d], b->stream, &rc, false);
    if (rc == LBM_OK) rc = init_kernels(b->views[d], phi0_dev[d], u0_dev ? u0_dev[d] : nullptr);
  }
  if (rc == LBM_OK && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
    rc = fail(LBM_EDEVICE, "stream create");
  if (rc == LBM_OK) {
    size_t maxn = 1;
    for (auto* v : b->views) maxn = std::max(maxn, v->N);
    b->ppd = reduce_ppd(maxn, ndom);
    hipError_t e = hipMalloc(&b->part, sizeof(double) * 2 * (size_t)ndom * b->ppd);
    if (e == hipSuccess) e = hipMalloc(&b->res, sizeof(double) * 2 * ndom);
    if (e == hipSuccess) e = hipHostMalloc(&b->res_host, sizeof(double) * 2 * ndom, hipHostMallocDefault);
    if (e != hipSuccess) rc = fail(LBM_ENOMEM, std::string("batch reduction scratch: ") + hipGetErrorString(e));
  }
  if (rc == LBM_OK) rc = scratch_on_current_device(&b->scratch);
  if (rc == LBM_OK) rc = batch_set_launch(b, 32, 8, 4, 0, true);
  if (rc) {
    lbm_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int n) {
  if (!b || n < 0) return fail(LBM_EINVAL, "bad handle or step count");
  if (n >= 2 && !b->g_pair) return fail(LBM_EINVAL, "no step graph (an autotune trial left the launch without one)");
  while (n > 0) {
    if ((b->steps & 1) || n == 1) {
      HIPCHK(launch_step(b->ls, b->Q, b->ST, (int)(b->steps & 1), b->stream));
      b->steps += 1;
      n -= 1;
    } else {
      HIPCHK(hipGraphLaunch(b->g_pair, b->stream));
      b->steps += 2;
      n -= 2;
    }
  }
  return LBM_OK;
}

long long lbm_batch_steps_done(const lbm_batch* b) { return b ? b->steps : -1; }

int lbm_batch_reduce(lbm_batch* b, double* mass, double* kinetic) {
  if (!b || !mass || !kinetic) return fail(LBM_EINVAL, "null argument");
  batch_sync_views(b);
  HIPCHK(launch_reduce(b->ls, b->Q, b->ST, (int)(b->steps & 1), b->ppd, b->part, b->res, b->stream));
  HIPCHK(hipMemcpyAsync(b->res_host, b->res, 2 * sizeof(double) * b->ndom, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  bool finite = true;
  for (int d = 0; d < b->ndom; ++d) {
    mass[d] = b->res_host[2 * d];
    kinetic[d] = b->res_host[2 * d + 1];
    finite = finite && std::isfinite(mass[d]) && std::isfinite(kinetic[d]);
  }
  if (!finite) return fail(LBM_EUNSTABLE, "non-finite mass or kinetic energy in a domain");
  return LBM_OK;
}

int lbm_batch_reduce_noalloc(lbm_batch* b, double* out_dev) {
  if (!b || !out_dev) return fail(LBM_EINVAL, "null argument");
  if (b->ndom > kReduceMaxParts)
    return fail(LBM_EINVAL, "lbm_batch_reduce_noalloc: at most " + std::to_string(kReduceMaxParts) +
                                " domains (the static scratch holds that many partial sums)");
  if ((size_t)b->ndom * b->ppd > (size_t)kReduceMaxParts)
    return fail(LBM_EINVAL, "lbm_batch_reduce_noalloc: partial sums exceed the static scratch");
  if (!b->scratch) return fail(LBM_EDEVICE, "static scratch address not resolved on this device");
  batch_sync_views(b);
  HIPCHK(launch_reduce(b->ls, b->Q, b->ST, (int)(b->steps & 1), b->ppd, b->scratch, out_dev, b->stream));
  return LBM_OK;
}

int lbm_batch_fields(lbm_batch* b, int dom, unsigned mask, float* phi_dev, float* u_dev, float* p_dev) {
  if (!b || dom < 0 || dom >= b->ndom) return fail(LBM_EINVAL, "bad handle or domain");
  batch_sync_views(b);
  return lbm_fields(b->views[dom], mask, phi_dev, u_dev, p_dev);
}

int lbm_batch_export_state(lbm_batch* b, int dom, float* h_dev, float* g_dev, float* u_dev) {
  if (!b || dom < 0 || dom >= b->ndom) return fail(LBM_EINVAL, "bad handle or domain");
  batch_sync_views(b);
  return lbm_export_state(b->views[dom], h_dev, g_dev, u_dev);
}

int lbm_batch_intact_length(lbm_batch* b, float threshold, int* length) {
  if (!b || !length) return fail(LBM_EINVAL, "null argument");
  batch_sync_views(b);
  int maxz = 0;
  for (auto* v : b->views) maxz = std::max(maxz, v->Q == 9 ? v->P.ny : v->P.nz);
  if (maxz > b->count_cap) {
    if (b->d_count) (void)hipFree(b->d_count);
    b->d_count = nullptr;
    HIPCHK(hipMalloc(&b->d_count, sizeof(int) * maxz));
    b->count_cap = maxz;
  }
  std::vector<int> cnt(maxz);
  for (int d = 0; d < b->ndom; ++d) {
    lbm_sim* v = b->views[d];
    HIPCHK(launch_phi(v));
    const int planes = v->Q == 9 ? v->P.ny : v->P.nz;
    hipLaunchKernelGGL(k_plane_count, dim3(planes), dim3(256), 0, b->stream, (const float*)v->out_buf(v->parity()),
                       v->K.plane, planes, threshold, b->d_count);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(cnt.data(), b->d_count, sizeof(int) * planes, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    int L = planes;
    for (int z = 0; z < planes; ++z)
      if (cnt[z] == 0) {
        L = z;
        break;
      }
    length[d] = L;
  }
  return LBM_OK;
}

int lbm_batch_set_launch(lbm_batch* b, int bx, int by, int blocks_per_cu, int nontemporal) {
  if (!b) return fail(LBM_EINVAL, "null handle");
  if (!tile_ok(bx, by) || blocks_per_cu < 0 || blocks_per_cu > 64) return fail(LBM_EINVAL, "bad launch shape");
  return batch_set_launch(b, bx, by, blocks_per_cu, nontemporal ? 1 : 0, true);
}

int lbm_batch_set_zchunk(lbm_batch* b, int planes) {
  if (!b || planes < 0 || planes > 4096) return fail(LBM_EINVAL, "bad argument");
  b->ls.zc = planes;
  return batch_set_launch(b, b->ls.bx, b->ls.by, b->ls.bpc, b->ls.nt, true);
}

int lbm_batch_autotune(lbm_batch* b, int trial_steps, int* bx, int* by, int* blocks_per_cu, int* nontemporal,
                       double* ms_per_step) {
  if (!b || trial_steps < 1) return fail(LBM_EINVAL, "bad argument");
  const std::string key = batch_key(b);
  TuneEntry best = {b->ls.bx, b->ls.by, b->ls.bpc, b->ls.nt, b->ls.zc, 1e30};
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      best = it->second;
      cached = true;
    }
  }
  if (!cached) {
    int w = b->views[0]->box.nx, miny = 1 << 30;
    for (auto* v : b->views) {
      if (v->box.nx != w) w = 0;
      miny = std::min(miny, v->P.ny);
    }
    for (const auto& cb : tile_candidates(w, miny)) {
      for (int bp : kBpc)
        for (int nt = 0; nt < 2; ++nt)
          for (int zc : kZc) {
            if (zc && b->Q != 19) continue;
            b->ls.zc = zc;
            int rc = batch_set_launch(b, cb.first, cb.second, bp, nt, false);
            double ms = 0.0;
            if (rc == LBM_OK) rc = time_steps(b->ls, b->Q, b->ST, b->stream, b->steps, 2, &ms);
            if (rc == LBM_OK) rc = time_steps(b->ls, b->Q, b->ST, b->stream, b->steps, trial_steps, &ms);
            if (rc) return rc;
            if (ms < best.ms) best = {cb.first, cb.second, bp, nt, zc, ms};
          }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  b->ls.zc = best.zc;
  int rc = batch_set_launch(b, best.bx, best.by, best.bpc, best.nt, true);
  if (rc) return rc;
  if (bx) *bx = best.bx;
  if (by) *by = best.by;
  if (blocks_per_cu) *blocks_per_cu = best.bpc;
  if (nontemporal) *nontemporal = best.nt;
  if (ms_per_step) *ms_per_step = best.ms;
  return LBM_OK;
}

int lbm_batch_kernel_times(lbm_batch* b, int n, double* out_ms) {
  if (!b || n < 1 || !out_ms) return fail(LBM_EINVAL, "bad argument");
  return phase_times(b->ls, b->Q, b->ST, b->stream, b->steps, n, out_ms);
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  drop_graph(b->g_pair);
  free_launch(b->ls);
  for (auto* v : b->views)
    if (v) lbm_destroy(v);
  if (b->d_count) (void)hipFree(b->d_count);
  if (b->part) (void)hipFree(b->part);
  if (b->res) (void)hipFree(b->res);
  if (b->res_host) (void)hipHostFree(b->res_host);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

}  // extern "C"
