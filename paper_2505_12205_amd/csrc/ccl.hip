// ccl.hip -- connected components of the liquid {phi > thr} and the
// per-component statistics of the drop-size diagnostic, for gfx950.
//
// Labelling is a lock-free union-find over the node array (labels only
// decrease, a root is linked to a smaller root with an atomic minimum, so
// every component ends labelled by its smallest node index):
//   k_init    each liquid node points at the start of its run along x within
//             its 64-lane wave (found with one ballot), so runs need no union;
//   k_merge   unions across wave seams along x, the periodic x seam, and the
//             lower y and z neighbours -- only where the left neighbours of
//             the pair are not both liquid, so each pair of overlapping runs
//             is joined once, at the start of its overlap;
//   k_flatten every liquid node takes its root.
// Statistics: the roots are compacted in ascending order (counts per chunk
// of 4096 nodes, one scan, ordered writes), then every run of equal labels
// within a wave adds its length and extent to a per-block table in LDS,
// flushed once per block.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>
#include <cmath>
#include <string>

#include "drops.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(DR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int TPB = 256;
constexpr int SLABS = 16;              // 256-node slabs per compaction block
constexpr int CHUNK = TPB * SLABS;     // nodes per compaction block
constexpr int UNION_CAP = 1 << 20;  // retries of one union; hitting it flags an error
constexpr int FIND_CAP = 1 << 26;   // steps of one root search (a chain strictly decreases)

struct Ext {
  int nx, ny, nz, N;
};

// labels are read through the device-coherent level: a root search must see
// the links other waves made
__device__ __forceinline__ int ld_label(const int* L, int i) {
  return __hip_atomic_load(L + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_root(const int* L, int x, int* flag) {
  int p = ld_label(L, x);
  for (int it = 0; p != x; ++it) {
    if (it >= FIND_CAP) {
      atomicOr(flag, 1);
      break;
    }
    x = p;
    p = ld_label(L, x);
  }
  return x;
}

// join the sets of a and b: link the larger root to the smaller one; if the
// larger was linked meanwhile, continue from its new parent
__device__ void unite(int* L, int a, int b, int* flag) {
  for (int it = 0; it < UNION_CAP; ++it) {
    a = find_root(L, a, flag);
    b = find_root(L, b, flag);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(L + b, a);
    if (old == b) return;
    b = old;
  }
  atomicOr(flag, 2);
}

__device__ __forceinline__ uint64_t lanes_upto(int lane) {  // bits 0..lane
  return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

__global__ void k_clear(int* w, int n) {
  if ((int)threadIdx.x < n) w[threadIdx.x] = 0;
}

__global__ __launch_bounds__(TPB) void k_init(const float* __restrict__ phi, Ext e, float thr, int* __restrict__ L) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < e.N;
  const bool fg = valid && phi[i] > thr;
  const int x = valid ? i % e.nx : 0;
  const uint64_t mfg = __ballot(fg);
  const bool prev = lane > 0 && ((mfg >> (lane - 1)) & 1ull);
  const uint64_t starts = __ballot(fg && (!prev || x == 0));
  if (!valid) return;
  if (!fg) {
    L[i] = -1;
    return;
  }
  const int s = 63 - __clzll(starts & lanes_upto(lane));  // this run's first lane
  L[i] = i - (lane - s);
}

__global__ __launch_bounds__(TPB) void k_merge(const float* __restrict__ phi, Ext e, unsigned per, float thr,
                                               int* L, int* flag) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i >= e.N || !(phi[i] > thr)) return;
  const int lane = threadIdx.x & 63;
  const int plane = e.nx * e.ny;
  const int x = i % e.nx, y = (i / e.nx) % e.ny, z = i / plane;
  const bool left = x > 0 && phi[i - 1] > thr;
  if (x > 0) {
    if (lane == 0 && left) unite(L, i, i - 1, flag);  // a run continued from the previous wave
  } else if ((per & 1u) && e.nx > 1 && phi[i + e.nx - 1] > thr) {
    unite(L, i, i + e.nx - 1, flag);
  }
  // lower neighbours along y and z (wrapping where periodic)
  int j = -1;
  if (y > 0) j = i - e.nx;
  else if ((per & 2u) && e.ny > 1) j = i + (e.ny - 1) * e.nx;
  if (j >= 0 && phi[j] > thr && !(left && phi[j - 1] > thr)) unite(L, i, j, flag);
  j = -1;
  if (z > 0) j = i - plane;
  else if ((per & 4u) && e.nz > 1) j = i + (e.nz - 1) * plane;
  if (j >= 0 && phi[j] > thr && !(left && phi[j - 1] > thr)) unite(L, i, j, flag);
}

__global__ __launch_bounds__(TPB) void k_flatten(Ext e, int* L, int* flag) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i >= e.N) return;
  const int l = L[i];
  if (l < 0) return;
  __hip_atomic_store(L + i, find_root(L, l, flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// roots per chunk of CHUNK nodes
__global__ __launch_bounds__(TPB) void k_root_count(const int* __restrict__ L, Ext e, int* __restrict__ cnt) {
  int r = 0;
  for (int s = 0; s < SLABS; ++s) {
    const int i = blockIdx.x * CHUNK + s * TPB + threadIdx.x;
    r += __syncthreads_count(i < e.N && L[i] == i);
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = r;
}

// exclusive scan of the block counts (one block of 1024 threads); total -> *ncomp
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ cnt, int nblk, int* __restrict__ off,
                                               int* __restrict__ ncomp) {
  __shared__ int s[1024];
  int carry = 0;
  for (int b0 = 0; b0 < nblk; b0 += 1024) {
    const int b = b0 + (int)threadIdx.x;
    const int v = b < nblk ? cnt[b] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
      const int t = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < nblk) off[b] = carry + s[threadIdx.x] - v;
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ncomp = carry;
}

// component index of every root, in ascending node order (the chunk's
// offset, then slab by slab); initialise the outputs
__global__ __launch_bounds__(TPB) void k_root_write(const int* __restrict__ L, Ext e, const int* __restrict__ off,
                                                    int cap, int* __restrict__ cid, int* __restrict__ root,
                                                    int* __restrict__ size, int* __restrict__ lo,
                                                    int* __restrict__ hi) {
  __shared__ int wcount[TPB / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int base = off[blockIdx.x];
  for (int s = 0; s < SLABS; ++s) {
    const int i = blockIdx.x * CHUNK + s * TPB + threadIdx.x;
    const bool isroot = i < e.N && L[i] == i;
    const uint64_t m = __ballot(isroot);
    if (lane == 0) wcount[wv] = __popcll(m);
    __syncthreads();
    int rank = __popcll(m & (lanes_upto(lane) >> 1));
    for (int w = 0; w < wv; ++w) rank += wcount[w];
    const int slab_total = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    if (isroot) {
      const int k = base + rank;
      cid[i] = k;
      if (k < cap) {
        root[k] = i;
        size[k] = 0;
        lo[k] = INT_MAX;
        hi[k] = -1;
      }
    }
    base += slab_total;
    __syncthreads();  // wcount is rewritten by the next slab
  }
}

// size and extent: every run of equal labels within a wave row adds its
// length and extent to its component's entry in a per-block LDS table (open
// addressing on the component index), which is added to the outputs once per
// block; a run whose probe finds no slot goes to the outputs directly
constexpr int ATAB = 128, APROBE = 8;

__global__ __launch_bounds__(TPB) void k_accumulate(const int* __restrict__ L, Ext e, int axis,
                                                    const int* __restrict__ cid, int cap, int* size, int* lo,
                                                    int* hi) {
  __shared__ int tk[ATAB], ts[ATAB], tlo[ATAB], thi[ATAB];
  for (int t = threadIdx.x; t < ATAB; t += TPB) {
    tk[t] = -1;
    ts[t] = 0;
    tlo[t] = INT_MAX;
    thi[t] = -1;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (int sl = 0; sl < SLABS; ++sl) {
    const int i = blockIdx.x * CHUNK + sl * TPB + threadIdx.x;
    const bool valid = i < e.N;
    const int l = valid ? L[i] : -1;
    const int lp = __shfl_up(l, 1);
    const int x = valid ? i % e.nx : 0;
    const bool fg = l >= 0;
    const bool start = fg && (lane == 0 || lp != l || x == 0);
    const uint64_t ms = __ballot(start);
    const uint64_t brk = ms | ~__ballot(fg);  // lanes that do not continue the lane before
    if (!start) continue;
    const uint64_t after = brk & ~lanes_upto(lane);
    const int end = after ? __ffsll((long long)after) - 2 : 63;  // last lane of this run
    const int len = end - lane + 1;
    const int k = cid[l];
    if (k >= cap) continue;
    int c;
    if (axis == 0) c = x;
    else if (axis == 1) c = (i / e.nx) % e.ny;
    else c = i / (e.nx * e.ny);
    const int chi = axis == 0 ? c + len - 1 : c;
    int slot = -1;
    for (int p = 0, h = k & (ATAB - 1); p < APROBE; ++p, h = (h + 1) & (ATAB - 1)) {
      const int old = atomicCAS(&tk[h], -1, k);
      if (old == -1 || old == k) {
        slot = h;
        break;
      }
    }
    if (slot >= 0) {
      atomicAdd(&ts[slot], len);
      atomicMin(&tlo[slot], c);
      atomicMax(&thi[slot], chi);
    } else {
      atomicAdd(size + k, len);
      atomicMin(lo + k, c);
      atomicMax(hi + k, chi);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ATAB; t += TPB) {
    const int k = tk[t];
    if (k < 0) continue;
    atomicAdd(size + k, ts[t]);
    atomicMin(lo + k, tlo[t]);
    atomicMax(hi + k, thi[t]);
  }
}

__global__ void k_deq(const int* __restrict__ ncomp, int cap, bool three_d, const int* __restrict__ size,
                      float* __restrict__ deq) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cap || k >= *ncomp) return;
  const float v = (float)size[k];
  deq[k] = three_d ? cbrtf(6.0f * v / 3.14159265358979f) : sqrtf(4.0f * v / 3.14159265358979f);
}

struct WsLayout {
  size_t flag, ncomp, cnt, off, cid, total;
  int nblk, nchunk;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool layout_of(int nx, int ny, int nz, WsLayout& w) {
  if (nx < 1 || ny < 1 || nz < 1) return false;
  const double n = (double)nx * ny * nz;
  if (n > (double)(1 << 30)) return false;
  const int N = nx * ny * nz;
  w.nblk = (N + TPB - 1) / TPB;
  w.nchunk = (N + CHUNK - 1) / CHUNK;
  w.flag = 0;
  w.ncomp = sizeof(int);
  w.cnt = 256;
  w.off = w.cnt + align256(sizeof(int) * (size_t)w.nchunk);
  w.cid = w.off + align256(sizeof(int) * (size_t)w.nchunk);
  w.total = w.cid + align256(sizeof(int) * (size_t)N);
  return true;
}

}  // namespace

extern "C" {

const char* dr_last_error(void) { return g_err.c_str(); }

size_t dr_workspace_bytes(int nx, int ny, int nz) {
  WsLayout w;
  return layout_of(nx, ny, nz, w) ? w.total : 0;
}

int dr_label(const float* phi, int nx, int ny, int nz, unsigned periodic, float thr, int* label, void* ws,
             size_t ws_bytes, void* stream) {
  WsLayout w;
  if (!layout_of(nx, ny, nz, w)) return fail(DR_EINVAL, "extent must be >= 1 per axis and at most 2^30 nodes");
  if (!phi || !label || !ws) return fail(DR_EINVAL, "null buffer");
  if (ws_bytes < w.total) return fail(DR_EINVAL, "workspace smaller than dr_workspace_bytes()");
  if (periodic & ~7u) return fail(DR_EINVAL, "periodic has bits beyond the three axes");
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  int* flag = (int*)(base + w.flag);
  const Ext e{nx, ny, nz, nx * ny * nz};
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, st, flag, 2);
  hipLaunchKernelGGL(k_init, dim3(w.nblk), dim3(TPB), 0, st, phi, e, thr, label);
  hipLaunchKernelGGL(k_merge, dim3(w.nblk), dim3(TPB), 0, st, phi, e, periodic, thr, label, flag);
  hipLaunchKernelGGL(k_flatten, dim3(w.nblk), dim3(TPB), 0, st, e, label, flag);
  HIPCHK(hipGetLastError());
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflag) return fail(DR_EINTERNAL, "union-find iteration bound exceeded");
  return DR_OK;
}

int dr_components(const int* label, int nx, int ny, int nz, int axis, int cap, int* root, int* size, int* lo,
                  int* hi, float* deq, int* ncomp, void* ws, size_t ws_bytes, void* stream) {
  WsLayout w;
  if (!layout_of(nx, ny, nz, w)) return fail(DR_EINVAL, "extent must be >= 1 per axis and at most 2^30 nodes");
  if (!label || !ws || !ncomp) return fail(DR_EINVAL, "null buffer");
  if (cap < 0 || (cap > 0 && (!root || !size || !lo || !hi || !deq))) return fail(DR_EINVAL, "bad outputs");
  if (axis < 0 || axis > 2) return fail(DR_EINVAL, "axis must be 0, 1 or 2");
  if (ws_bytes < w.total) return fail(DR_EINVAL, "workspace smaller than dr_workspace_bytes()");
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  int* nc = (int*)(base + w.ncomp);
  int* cnt = (int*)(base + w.cnt);
  int* off = (int*)(base + w.off);
  int* cid = (int*)(base + w.cid);
  const Ext e{nx, ny, nz, nx * ny * nz};
  hipLaunchKernelGGL(k_root_count, dim3(w.nchunk), dim3(TPB), 0, st, label, e, cnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, w.nchunk, off, nc);
  hipLaunchKernelGGL(k_root_write, dim3(w.nchunk), dim3(TPB), 0, st, label, e, off, cap, cid, root, size, lo,
                     hi);
  hipLaunchKernelGGL(k_accumulate, dim3(w.nchunk), dim3(TPB), 0, st, label, e, axis, cid, cap, size, lo, hi);
  if (cap > 0)
    hipLaunchKernelGGL(k_deq, dim3((cap + 255) / 256), dim3(256), 0, st, nc, cap, nz > 1, size, deq);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(ncomp, nc, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (*ncomp > cap) return fail(DR_ECAPACITY, "more components than the capacity");
  return DR_OK;
}

}  // extern "C"
