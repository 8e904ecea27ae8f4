// nn.hip -- gfx950 kernels of the learned surrogate (include/surrogate.h).
//
// The convolutions are implicit GEMMs on the bf16 matrix cores (FP32
// accumulation; v_mfma_f32_16x16x32_bf16 for the forward and data gradient,
// v_mfma_f32_16x16x16_bf16 for the weight gradient):
//   forward      M = output voxels, N = co, K = 27 taps x ci
//   data grad    M = input voxels,  N = ci, K = 27 taps x (up^3 sub-positions) x co
//   weight grad  M = co, N = ci (one tap per block row), K = output voxels
// Activations are NDHWC bf16 with 16 | C, so every lane reads its operand
// values (8 consecutive K entries: channels of one tap) with one 16-byte
// load.  A wave owns 16*MS voxels x 16*NS channels with
// MS * NS = 8 accumulator tiles.  The weight gradient stages 64-voxel tiles
// of dz and of the gathered input in LDS, transposed so that the voxel
// (reduction) index is contiguous.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>

#include "surrogate.h"

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return SG_OK;
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// float -> bf16 rounded to nearest even: gfx950's conversion instruction
// (v_cvt_pk_bf16_f32), two values per instruction in f2bf2
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, (v2bf){(__bf16)lo, (__bf16)hi});
}
__device__ __forceinline__ uint4 f2bf8(const float (&v)[8]) {
  return (uint4){f2bf2(v[0], v[1]), f2bf2(v[2], v[3]), f2bf2(v[4], v[5]), f2bf2(v[6], v[7])};
}

__device__ __forceinline__ v4s ld4(const uint16_t* p) { return *(const v4s*)p; }

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// gfx950's 16 x 16 x 32 form: every lane holds 8 consecutive K values of its
// A row and of its B column (K index 8 (lane / 16) + j), D as above
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8u __attribute__((ext_vector_type(8)));  // 8 bf16 bit patterns
__device__ __forceinline__ v8bf ld8(const uint16_t* p) { return *(const v8bf*)p; }
__device__ __forceinline__ v4f mfma32(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

struct Geo {
  int n, d, h, w;    // layer input extent
  int ci, co;        // channels
  int od, oh, ow;    // layer output extent
  long long mi, mo;  // input / output voxels over the batch
};

Geo make_geo(int n, int d, int h, int w, int ci, int co, int s, int u) {
  Geo g;
  g.n = n;
  g.d = d;
  g.h = h;
  g.w = w;
  g.ci = ci;
  g.co = co;
  g.od = (u * d + s - 1) / s;
  g.oh = (u * h + s - 1) / s;
  g.ow = (u * w + s - 1) / s;
  g.mi = (long long)n * d * h * w;
  g.mo = (long long)n * g.od * g.oh * g.ow;
  return g;
}

// ---------------------------------------------------------------------------
// epilogues: accumulators staged in LDS, written 16 bytes per lane
// ---------------------------------------------------------------------------
// A wave's accumulators (lane: D[4 quad + r][col] of row tile m and channel
// tile s) are staged in LDS as FP32 [16 MS voxels][16 NS channels]; every
// lane then takes 8 consecutive channels of one voxel, so the global
// accesses (add, mask, da, dzp) are 16 bytes per lane.  vox(m, xl) is the
// global voxel of the wave's voxel xl in row m, or -1 outside the grid.
template <int MS, int NS>
__device__ __forceinline__ void stage_acc(float* stage, const v4f (&acc)[MS][NS], int quad, int col) {
  constexpr int CW = 16 * NS;
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int r = 0; r < 4; ++r) stage[(m * 16 + 4 * quad + r) * CW + s * 16 + col] = acc[m][s][r];
}

template <int MS, int NS, class Vox>
__device__ __forceinline__ void dgrad_epilogue(const float* stage, int lane, Vox vox,
                                               const uint16_t* __restrict__ add,
                                               const uint16_t* __restrict__ mask, uint16_t* __restrict__ da,
                                               uint16_t* __restrict__ dzp) {
  constexpr int CW = 16 * NS, G = CW / 8, VOX = 16 * MS;
#pragma unroll
  for (int j = 0; j < VOX * G / 64; ++j) {
    const int f = j * 64 + lane, vl = f / G, c0 = (f % G) * 8;
    const long long v = vox(vl / 16, vl % 16);
    if (v < 0) continue;
    const long long i = v * CW + c0;
    const v4f lo = *(const v4f*)&stage[vl * CW + c0], hi = *(const v4f*)&stage[vl * CW + c0 + 4];
    v8u av = {}, mv = {};
    float od[8], oz[8];
    if (add) av = *(const v8u*)(add + i);
    if (mask) mv = *(const v8u*)(mask + i);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float val = e < 4 ? lo[e] : hi[e - 4];
      if (add) val += bf2f(av[e]);
      od[e] = val;
      if (mask && !(bf2f(mv[e]) > 0.0f)) val = 0.0f;
      oz[e] = val;
    }
    if (da) *(uint4*)(da + i) = f2bf8(od);
    *(uint4*)(dzp + i) = f2bf8(oz);
  }
}

// ---------------------------------------------------------------------------
// forward: y[v, o] = act(b[o] + sum_{k,c} w[o,k,c] X[src(v,k), c]) (+ skip)
// ---------------------------------------------------------------------------
template <int CO, int S, int U>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ wgt,
                                                  const float* __restrict__ bias,
                                                  const uint16_t* __restrict__ skip, uint16_t* __restrict__ y,
                                                  uint16_t* __restrict__ yr, Geo g, int relu) {
  constexpr int NS = CO / 16;
  constexpr int MS = 8 / NS;
  __shared__ __attribute__((aligned(16))) float fw_stage[4 * 16 * MS * CO];  // the epilogue's staging
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const long long vbase = ((long long)blockIdx.x * 4 + wv) * (16 * MS);
  int pz[MS], py[MS], px[MS], nb[MS];
  bool ok[MS];
#pragma unroll
  for (int m = 0; m < MS; ++m) {
    long long v = vbase + m * 16 + col;  // A row of this lane
    ok[m] = v < g.mo;
    if (!ok[m]) v = 0;
    px[m] = (int)(v % g.ow);
    v /= g.ow;
    py[m] = (int)(v % g.oh);
    v /= g.oh;
    pz[m] = (int)(v % g.od);
    nb[m] = (int)(v / g.od);
  }
  v4f acc[MS][NS];
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[m][s] = (v4f){0.f, 0.f, 0.f, 0.f};
  const v8bf zero = {};
  const int DU = g.d * U, HU = g.h * U, WU = g.w * U;
  // K = 27 taps x ci, tap-major; a 32-wide K chunk gives each lane 8
  // channels of one tap (16 | ci)
  const int K = 27 * g.ci, csh = ilog2(g.ci);
  // The chunk's weight tile (CO rows of 32 K values, row o at wgt + o K + k0,
  // zero past K) is loaded once per block into a double-buffered LDS tile
  // (rows padded to 40 elements: a 16-lane read of 16 bytes from 16 rows hits
  // distinct banks) instead of once per wave; the epilogue's staging buffer
  // holds it during the K loop.
  constexpr int WR = 40;
  static_assert(2 * CO * WR * 2 <= (int)sizeof(fw_stage), "weight tiles fit the staging buffer");
  uint16_t* wl = (uint16_t*)fw_stage;
  const int wt = threadIdx.x;  // thread wt < 4 CO loads 8 K values of row wt / 4
  auto wload = [&](int k0) {
    uint4 v = {0u, 0u, 0u, 0u};
    const int k = k0 + (wt & 3) * 8;  // K is a multiple of 16: 8 values are all in or all out
    if (wt < 4 * CO && k < K) v = *(const uint4*)(wgt + (long long)(wt >> 2) * K + k);
    return v;
  };
  auto wstore = [&](int buf, uint4 v) {
    if (wt < 4 * CO) *(uint4*)&wl[(buf * CO + (wt >> 2)) * WR + (wt & 3) * 8] = v;
  };
  auto load = [&](int k0, v8bf* a) {
    const int k = k0 + 8 * quad;
    const bool kin = k < K;
    const int tap = kin ? (k >> csh) : 0, c = k - (tap << csh);
    const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
#pragma unroll
    for (int m = 0; m < MS; ++m) {
      const int qz = pz[m] * S + kz - 1, qy = py[m] * S + ky - 1, qx = px[m] * S + kx - 1;
      const bool in = kin && ok[m] && qz >= 0 && qz < DU && qy >= 0 && qy < HU && qx >= 0 && qx < WU;
      a[m] = in ? ld8(x + ((((long long)nb[m] * g.d + qz / U) * g.h + qy / U) * g.w + qx / U) * g.ci + c)
                : zero;
    }
  };
  const int nch = (K + 31) / 32;
  uint4 wn = wload(0);
  wstore(0, wn);
  if (nch > 1) wn = wload(32);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int k0 = ch * 32, buf = ch & 1;
    v8bf a[MS], b[NS];
    load(k0, a);
#pragma unroll
    for (int s = 0; s < NS; ++s) b[s] = *(const v8bf*)&wl[(buf * CO + s * 16 + col) * WR + 8 * quad];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int m = 0; m < MS; ++m) acc[m][s] = mfma32(a[m], b[s], acc[m][s]);
    if (ch + 1 < nch) {
      wstore(buf ^ 1, wn);  // the other tile's readers passed the previous barrier
      if (ch + 2 < nch) wn = wload(k0 + 64);
    }
    __syncthreads();
  }
  // lane holds D[4 quad + r][col]: voxel row 4 quad + r, channel col; staged
  // in LDS, then written 8 channels of one voxel per lane (16-byte accesses)
  float* stage = fw_stage + wv * (16 * MS) * CO;
  stage_acc<MS, NS>(stage, acc, quad, col);
  __syncthreads();
  constexpr int G = CO / 8;
#pragma unroll
  for (int j = 0; j < 16 * MS * G / 64; ++j) {
    const int f = j * 64 + lane, vl = f / G, c0 = (f % G) * 8;
    const long long v = vbase + vl;
    if (v >= g.mo) continue;
    const long long i = v * CO + c0;
    const v4f lo = *(const v4f*)&stage[vl * CO + c0], hi = *(const v4f*)&stage[vl * CO + c0 + 4];
    v8u sv = {};
    float orr[8], oy[8];
    if (skip) sv = *(const v8u*)(skip + i);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float val = (e < 4 ? lo[e] : hi[e - 4]) + bias[c0 + e];
      if (relu) val = fmaxf(val, 0.0f);
      orr[e] = val;
      if (skip) val += bf2f(sv[e]);
      oy[e] = val;
    }
    if (yr) *(uint4*)(yr + i) = f2bf8(orr);
    *(uint4*)(y + i) = f2bf8(oy);
  }
}

// Work item of block b of nb when consecutive blocks are dealt round-robin to
// the 8 XCDs: the blocks of one XCD take consecutive items (a tail of fewer
// than 8 blocks keeps its own index), so the halos that neighbouring tiles
// share are read while they are in that XCD's L2.
__device__ __forceinline__ int xcd_item(int b, int nb) {
  const int full = nb & ~7;
  return b >= full ? b : (b & 7) * (full >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// stride-1 convolution from an LDS halo tile (C channels in and out)
// ---------------------------------------------------------------------------
// A block owns TZ x TY rows of 16 output voxels along x; it stages the
// input brick with a one-voxel halo in LDS once, and every tap reads a
// shifted window of it.  With nearest upsampling (U = 2) the brick is staged
// at the input's resolution, (TZ/2 + 2) x (TY/2 + 2) x 10 voxels, and the
// tap at virtual position q reads staged voxel floor(q / 2).  MODE 0 is the forward epilogue (bias, relu, the activation
// before the skip in y2, skip add); MODE 1 is the data gradient of a stride-1
// layer (U = 1, CI = CO): with the flipped weights wf[c][26 - k][o] =
// w[o][k][c] the gradient is the same convolution of dz, and the epilogue
// adds `add`, stores the sum in y2 and the sum masked by mask > 0 in y.
template <int CI, int CO, int U>
struct HaloTile {
  static constexpr int NS = CO / 16, MS = 8 / NS, ROWS = 4 * MS;
  static constexpr int TY = ROWS >= 16 ? 8 : 4, TZ = ROWS / TY;
  static constexpr int HX = U == 1 ? 18 : 10, HY = U == 1 ? TY + 2 : TY / 2 + 2, HZ = U == 1 ? TZ + 2 : TZ / 2 + 2;
  static constexpr int ELEMS = HZ * HY * HX * CI;
  // the tiles whose waves split the channels are held to two waves per
  // SIMD's registers
  static constexpr int WPE = U == 1 && NS >= 2 ? 2 : 1;
};

struct HGeo {
  int n, d, h, w;          // input extent
  int od, oh, ow;          // output extent (U x input)
  int ntx, nty, ntz;       // tiles along x, y, z
};

template <int CI, int CO, int U, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HaloTile<CI, CO, U>::WPE))) void k_conv_halo(const uint16_t* __restrict__ x, const uint16_t* __restrict__ wgt,
                                                   const float* __restrict__ bias,
                                                   const uint16_t* __restrict__ other,
                                                   const uint16_t* __restrict__ mask, uint16_t* __restrict__ y,
                                                   uint16_t* __restrict__ y2, HGeo g, int relu) {
  using T = HaloTile<CI, CO, U>;
  constexpr int NS = T::NS, MS = T::MS, TY = T::TY, TZ = T::TZ, HX = T::HX, HY = T::HY, HZ = T::HZ;
  // the halo, then (after the K loop) the epilogue's FP32 staging of the
  // four waves' accumulators: the larger of the two
  constexpr int STAGE_ELEMS = 4 * 16 * MS * 16 * NS * 2;
  __shared__ __attribute__((aligned(16))) uint16_t halo[T::ELEMS > STAGE_ELEMS ? T::ELEMS : STAGE_ELEMS];
  int b = xcd_item(blockIdx.x, gridDim.x);
  const int tx = b % g.ntx;
  b /= g.ntx;
  const int ty = b % g.nty;
  b /= g.nty;
  const int tz = b % g.ntz;
  const int n = b / g.ntz;
  const int x0 = tx * 16, y0 = ty * TY, z0 = tz * TZ;
  // stage the brick and its halo, zero outside the grid; the staged origin
  // is one input voxel before the brick (x0, y0, z0 are even for U = 2).
  // Every load of a thread is issued before the first LDS write.  Item i is
  // 8 channels of one staged voxel, row-major over the staged rows of HX
  // voxels; its global offset is that of the staged origin plus the row's
  // and the voxel's.
  constexpr int CG = CI / 8, RW = HX * CG, NITEMS = HZ * HY * RW, PT = (NITEMS + 255) / 256;
  const int sz0 = z0 / U - 1, sy0 = y0 / U - 1, sx0 = x0 / U - 1;
  const long long obase = (((long long)n * g.d + sz0) * g.h + sy0) * g.w + sx0;  // may lie before x: offset only
  v8bf val[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int row = i / RW, e = i - row * RW, hz = row / HY, hy = row - hz * HY, hx = e / CG;
    const bool in = (NITEMS % 256 == 0 || i < NITEMS) && (unsigned)(sz0 + hz) < (unsigned)g.d &&
                    (unsigned)(sy0 + hy) < (unsigned)g.h && (unsigned)(sx0 + hx) < (unsigned)g.w;
    val[k] = (v8bf){};
    if (in) val[k] = ld8(x + (obase + (long long)(hz * g.h + hy) * g.w + hx) * CI + (e - hx * CG) * 8);
  }
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (NITEMS % 256 == 0 || i < NITEMS) *(v8bf*)&halo[i * 8] = val[k];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  // With 32 or 64 output channels the waves split the channels:
  // wave wv takes the 16-channel slice wv % NS over MS NS rows of the tile,
  // so it loads 1/NS of the weights per K chunk instead of all of them;
  // otherwise a wave takes MS rows and every channel.
  constexpr bool WS = NS >= 2;
  constexpr int MW = WS ? MS * NS : MS, NW = WS ? 1 : NS;  // a wave's rows and channel tiles
  v4f acc[MW][NW];
#pragma unroll
  for (int m = 0; m < MW; ++m)
#pragma unroll
    for (int s = 0; s < NW; ++s) acc[m][s] = (v4f){0.f, 0.f, 0.f, 0.f};
  constexpr int K = 27 * CI;
  constexpr int csh = CI == 16 ? 4 : (CI == 32 ? 5 : 6);
  if constexpr (U == 1) {
    // A wave's MS rows are MS consecutive y rows of one z plane, so the
    // staged voxel of row m and tap (kz, ky, kx) is that of row 0 plus
    // m * HX (a compile-time stride: an immediate LDS offset) plus the tap's
    // offset, which depends only on the K chunk and the lane's quad.  The
    // tap offsets of the chunk are wave-uniform; the lane picks one of two.
    static_assert(WS || TY % MS == 0, "a wave's rows lie in one z plane");
    const int r0 = WS ? (wv / NS) * MW : wv * MS;
    const int abase = (((r0 / TY) * HY + r0 % TY) * HX + col) * CI;
    // staged offset of the wave's row m from its row 0 (compile-time)
    auto row_off = [](int m) { return WS ? ((m / TY) * HY + m % TY) * HX * CI : m * HX * CI; };
    const uint16_t* wrow[NW];
#pragma unroll
    for (int s = 0; s < NW; ++s) wrow[s] = wgt + (long long)((WS ? wv % NS : s) * 16 + col) * K;
    auto tap_off = [](int t) { return (((t / 9) * HY + (t / 3) % 3) * HX + t % 3) * CI; };
    auto chunk = [&](int k0, bool tail) {
      const int k = k0 + 8 * quad;
      const bool kin = !tail || k < K;
      const int t0 = k0 >> csh;  // tap of quad 0 (uniform)
      const int o0 = tap_off(t0), o1 = tap_off(t0 + 1);
      const int c = kin ? k - (t0 << csh) : 0;  // < 2 CI: past CI the lane's tap is t0 + 1
      const int toff = (CI == 16 && c >= CI) ? o1 + (c - CI) : o0 + c;
      v8bf a[MW], bb[NW];
#pragma unroll
      for (int m = 0; m < MW; ++m)
        a[m] = kin ? *(const v8bf*)&halo[abase + toff + row_off(m)] : (v8bf){};
#pragma unroll
      for (int s = 0; s < NW; ++s) bb[s] = kin ? ld8(wrow[s] + k) : (v8bf){};
#pragma unroll
      for (int s = 0; s < NW; ++s)
#pragma unroll
        for (int m = 0; m < MW; ++m) acc[m][s] = mfma32(a[m], bb[s], acc[m][s]);
    };
    if constexpr (WS) {
      // one weight load per chunk: a rolled loop with the next D chunks'
      // weights in flight (a full unroll hoists the LDS reads into spills)
      constexpr int D = 3, NCH = K / 32;
      static_assert(CI >= 32 && NCH % D == 0, "chunks within one tap, whole groups of D");
      v8bf wq[D];
#pragma unroll
      for (int d = 0; d < D; ++d) wq[d] = ld8(wrow[0] + d * 32 + 8 * quad);
      for (int kb = 0; kb < NCH; kb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int k0 = (kb + d) * 32, t0 = k0 >> csh;
          const int toff = tap_off(t0) + (k0 - (t0 << csh)) + 8 * quad;
          v8bf a[MW];
#pragma unroll
          for (int m = 0; m < MW; ++m) a[m] = *(const v8bf*)&halo[abase + toff + row_off(m)];
#pragma unroll
          for (int m = 0; m < MW; ++m) acc[m][0] = mfma32(a[m], wq[d], acc[m][0]);
          if (kb + D < NCH) wq[d] = ld8(wrow[0] + k0 + D * 32 + 8 * quad);
        }
      }
    } else {
      constexpr int KF = K / 32 * 32;  // full chunks; CI = 16 leaves a half chunk
#pragma unroll
      for (int k0 = 0; k0 < KF; k0 += 32) chunk(k0, false);
      if constexpr (KF < K) chunk(KF, true);
    }
  } else {
    // x2 upsampling: the staged voxel of virtual offset t = row/col + tap - 1
    // is floor(t / 2) + 1 along each axis.  With at least 32 input channels a
    // 32-wide K chunk lies in one tap, and a wave's rows lie in one z plane,
    // so the tap, the staged plane and each row's staged row are
    // wave-uniform (scalar); a lane adds only its staged x voxel and
    // channels.
    static_assert(CI >= 32 && TY % MW == 0, "uniform taps and planes per wave");
    const int wu = __builtin_amdgcn_readfirstlane(wv);
    const int r0 = WS ? (wu / NS) * MW : wu * MS;
    const int rz = r0 / TY, ry0 = r0 % TY;
    const uint16_t* wrow[NW];
#pragma unroll
    for (int s = 0; s < NW; ++s) wrow[s] = wgt + (long long)((WS ? wu % NS : s) * 16 + col) * K + 8 * quad;
    // the weights of the next D chunks are in flight while a chunk multiplies
    constexpr int D = 3, NCH = K / 32;
    static_assert(NCH % D == 0, "whole groups of D chunks");
    v8bf wq[D][NW];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
      for (int s = 0; s < NW; ++s) wq[d][s] = ld8(wrow[s] + d * 32);
    for (int kb = 0; kb < NCH; kb += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int k0 = (kb + d) * 32;
        const int tap = k0 >> csh, c0 = k0 - (tap << csh);
        const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
        const int lz = ((rz + kz - 1) >> 1) + 1;
        const int xoff = (((col + kx - 1) >> 1) + 1) * CI + c0 + 8 * quad;
        v8bf a[MW];
#pragma unroll
        for (int m = 0; m < MW; ++m) {
          const int ly = ((ry0 + m + ky - 1) >> 1) + 1;
          a[m] = *(const v8bf*)&halo[(lz * HY + ly) * HX * CI + xoff];
        }
#pragma unroll
        for (int s = 0; s < NW; ++s)
#pragma unroll
          for (int m = 0; m < MW; ++m) acc[m][s] = mfma32(a[m], wq[d][s], acc[m][s]);
        if (kb + D < NCH)
#pragma unroll
          for (int s = 0; s < NW; ++s) wq[d][s] = ld8(wrow[s] + k0 + D * 32);
      }
    }
  }
  // lane holds D[4 quad + r][col]: voxel x0 + 4 quad + r of row m, channel s*16 + col
  // (row r0 + m and channel (wv % NS)*16 + col when the waves split the channels)
  constexpr int VOX = WS ? 16 * 4 * MS : 16 * MS, CW = 16 * NS;  // voxels and channels of a staging group
  constexpr int GT = WS ? 256 : 64;  // threads of a staging group: the block, or one wave
  // Stage the accumulators through the halo's LDS (the halo is no longer
  // read), then give every lane 8 consecutive channels of one voxel: the
  // epilogue's global accesses become 16 bytes per lane, contiguous across
  // lanes, instead of 2 bytes per lane in 32-byte pieces.
  __syncthreads();
  float* stage = (float*)halo + (WS ? 0 : wv * VOX * CW);
#pragma unroll
  for (int m = 0; m < MW; ++m)
#pragma unroll
    for (int s = 0; s < NW; ++s)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        stage[(((WS ? (wv / NS) * MW : 0) + m) * 16 + 4 * quad + r) * CW + (WS ? wv % NS : s) * 16 + col] =
            acc[m][s][r];
  __syncthreads();
  constexpr int G = CW / 8;  // 8-channel groups per voxel
  const int gi = WS ? (int)threadIdx.x : lane;
#pragma unroll
  for (int j = 0; j < VOX * G / GT; ++j) {
    const int f = j * GT + gi, vl = f / G, c0 = (f % G) * 8;
    const int m = vl / 16, xl = vl % 16;
    const int rr = (WS ? 0 : wv * MS) + m, gz = z0 + rr / TY, gy = y0 + rr % TY, gx = x0 + xl;
    if (gz >= g.od || gy >= g.oh || gx >= g.ow) continue;
    const long long i = ((((long long)n * g.od + gz) * g.oh + gy) * g.ow + gx) * CO + c0;
    const v4f lo = *(const v4f*)&stage[vl * CW + c0], hi = *(const v4f*)&stage[vl * CW + c0 + 4];
    v8u ov = {}, mv = {};
    float o2[8], oy[8];
    if (other) ov = *(const v8u*)(other + i);
    if (MODE == 1 && mask) mv = *(const v8u*)(mask + i);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float v = e < 4 ? lo[e] : hi[e - 4];
      if (MODE == 0) {
        v += bias[c0 + e];
        if (relu) v = fmaxf(v, 0.0f);
        o2[e] = v;
        if (other) v += bf2f(ov[e]);
      } else {
        if (other) v += bf2f(ov[e]);
        o2[e] = v;
        if (mask && !(bf2f(mv[e]) > 0.0f)) v = 0.0f;
      }
      oy[e] = v;
    }
    if (y2) *(uint4*)(y2 + i) = f2bf8(o2);
    *(uint4*)(y + i) = f2bf8(oy);
  }
}

// ---------------------------------------------------------------------------
// data gradient: g[r, c] = sum over (k, p) with src(p, k) = r of w[o,k,c] dz[p, o]
// ---------------------------------------------------------------------------
template <int CI, int S, int U>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const uint16_t* __restrict__ dz,
                                                       const uint16_t* __restrict__ wf, Geo g,
                                                       const uint16_t* __restrict__ add,
                                                       const uint16_t* __restrict__ mask,
                                                       uint16_t* __restrict__ da, uint16_t* __restrict__ dzp) {
  constexpr int NS = CI / 16;
  constexpr int MS = 8 / NS;
  __shared__ __attribute__((aligned(16))) float dg_stage[4 * 16 * MS * CI];  // the epilogue's staging
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const long long vbase = ((long long)blockIdx.x * 4 + wv) * (16 * MS);
  int rz[MS], ry[MS], rx[MS], nb[MS];
  bool ok[MS];
#pragma unroll
  for (int m = 0; m < MS; ++m) {
    long long v = vbase + m * 16 + col;
    ok[m] = v < g.mi;
    if (!ok[m]) v = 0;
    rx[m] = (int)(v % g.w);
    v /= g.w;
    ry[m] = (int)(v % g.h);
    v /= g.h;
    rz[m] = (int)(v % g.d);
    nb[m] = (int)(v / g.d);
  }
  v4f acc[MS][NS];
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[m][s] = (v4f){0.f, 0.f, 0.f, 0.f};
  const v8bf zero = {};
  // K = 27 taps x U^3 sub-positions x co; a 32-wide chunk gives each lane 8
  // channels of one (tap, sub-position) (16 | co)
  constexpr int U3 = U * U * U;
  const int K = 27 * U3 * g.co, osh = ilog2(g.co);
  auto load = [&](int k0, v8bf* a, v8bf* b) {
    const int k = k0 + 8 * quad;
    const bool kin = k < K;
    const int tj = kin ? (k >> osh) : 0, o = k - (tj << osh);
    const int tap = tj / U3, j = tj % U3;
    const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
    const int jz = j / (U * U), jy = (j / U) % U, jx = j % U;
#pragma unroll
    for (int m = 0; m < MS; ++m) {
      // virtual input position q = r U + j is read by output p when s p + k - 1 = q
      const int tz = rz[m] * U + jz + 1 - kz, ty = ry[m] * U + jy + 1 - ky, tx = rx[m] * U + jx + 1 - kx;
      bool v = kin && ok[m] && tz >= 0 && ty >= 0 && tx >= 0;
      if (S == 2) v = v && !(tz & 1) && !(ty & 1) && !(tx & 1);
      const int ppz = tz / S, ppy = ty / S, ppx = tx / S;
      v = v && ppz < g.od && ppy < g.oh && ppx < g.ow;
      a[m] = v ? ld8(dz + ((((long long)nb[m] * g.od + ppz) * g.oh + ppy) * g.ow + ppx) * g.co + o) : zero;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
      b[s] = kin ? ld8(wf + ((long long)(s * 16 + col) * 27 + (26 - tap)) * g.co + o) : zero;
  };
  for (int k0 = 0; k0 < K; k0 += 32) {
    v8bf a[MS], b[NS];
    load(k0, a, b);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int m = 0; m < MS; ++m) acc[m][s] = mfma32(a[m], b[s], acc[m][s]);
  }
  float* stage = dg_stage + wv * (16 * MS) * CI;
  stage_acc<MS, NS>(stage, acc, quad, col);
  __syncthreads();
  dgrad_epilogue<MS, NS>(stage, lane, [&](int m, int xl) -> long long {
    const long long v = vbase + m * 16 + xl;
    return v < g.mi ? v : -1;
  }, add, mask, da, dzp);
}

// ---------------------------------------------------------------------------
// data gradient of a x2 upsampling layer with folded weights
// ---------------------------------------------------------------------------
// Along each axis the upsampled position 2 r + j (j = 0, 1) of input voxel r
// is read by output p = 2 r + j + 1 - k, so over j and the taps k the
// outputs p = 2 r - 1 + a (a = 0..3) reach r, each through the taps of the
// fold set F(a) = [max(0, 2 - a), min(2, 3 - a)] ({2}, {1, 2}, {0, 1}, {0}).
// With wu[c][a][o] = sum over k in F(az) x F(ay) x F(ax) of w[o][k][c]
// (k_fold_up_w) the gradient is a 4 x 4 x 4 gather over dz with stride 2:
// K = 64 co instead of the 27 x 8 co of the gather over taps and
// sub-positions.
template <int CI>
__global__ __launch_bounds__(256) void k_conv_bwd_data_up2(const uint16_t* __restrict__ dz,
                                                           const uint16_t* __restrict__ wu, Geo g,
                                                           const uint16_t* __restrict__ add,
                                                           const uint16_t* __restrict__ mask,
                                                           uint16_t* __restrict__ da, uint16_t* __restrict__ dzp) {
  constexpr int NS = CI / 16;
  constexpr int MS = 8 / NS;
  __shared__ __attribute__((aligned(16))) float dg_stage[4 * 16 * MS * CI];  // the epilogue's staging
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const long long vbase = ((long long)blockIdx.x * 4 + wv) * (16 * MS);
  int pz0[MS], py0[MS], px0[MS], nb[MS];
  bool ok[MS];
#pragma unroll
  for (int m = 0; m < MS; ++m) {
    long long v = vbase + m * 16 + col;
    ok[m] = v < g.mi;
    if (!ok[m]) v = 0;
    px0[m] = 2 * (int)(v % g.w) - 1;
    v /= g.w;
    py0[m] = 2 * (int)(v % g.h) - 1;
    v /= g.h;
    pz0[m] = 2 * (int)(v % g.d) - 1;
    nb[m] = (int)(v / g.d);
  }
  v4f acc[MS][NS];
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[m][s] = (v4f){0.f, 0.f, 0.f, 0.f};
  const v8bf zero = {};
  const int K = 64 * g.co, osh = ilog2(g.co);  // a multiple of 32: no partial chunk
  // The chunk's weight tile (CI rows of 32 K values, row c at wu + c K + k0)
  // is loaded once per block into a double-buffered LDS tile (rows padded to
  // 40 elements: a 16-lane read of 16 bytes from 16 rows hits distinct
  // banks) instead of once per wave; the epilogue's staging buffer holds it
  // during the K loop.
  constexpr int WR = 40;
  static_assert(2 * CI * WR * 2 <= (int)sizeof(dg_stage), "weight tiles fit the staging buffer");
  uint16_t* wl = (uint16_t*)dg_stage;
  const int wt = threadIdx.x;  // thread wt < 4 CI loads 8 K values of row wt / 4
  auto wload = [&](int k0) {
    uint4 v = {0u, 0u, 0u, 0u};
    if (wt < 4 * CI) v = *(const uint4*)(wu + (long long)(wt >> 2) * K + k0 + (wt & 3) * 8);
    return v;
  };
  auto wstore = [&](int buf, uint4 v) {
    if (wt < 4 * CI) *(uint4*)&wl[(buf * CI + (wt >> 2)) * WR + (wt & 3) * 8] = v;
  };
  const int nch = K / 32;
  uint4 wn = wload(0);
  wstore(0, wn);
  if (nch > 1) wn = wload(32);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int k0 = ch * 32, buf = ch & 1;
    const int k = k0 + 8 * quad;
    const int t = k >> osh, o = k - (t << osh);
    const int az = t >> 4, ay = (t >> 2) & 3, ax = t & 3;
    v8bf a[MS], b[NS];
#pragma unroll
    for (int m = 0; m < MS; ++m) {
      const int pz = pz0[m] + az, py = py0[m] + ay, px = px0[m] + ax;
      const bool v = ok[m] && pz >= 0 && py >= 0 && px >= 0 && pz < g.od && py < g.oh && px < g.ow;
      a[m] = v ? ld8(dz + ((((long long)nb[m] * g.od + pz) * g.oh + py) * g.ow + px) * g.co + o) : zero;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) b[s] = *(const v8bf*)&wl[(buf * CI + s * 16 + col) * WR + 8 * quad];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int m = 0; m < MS; ++m) acc[m][s] = mfma32(a[m], b[s], acc[m][s]);
    if (ch + 1 < nch) {
      wstore(buf ^ 1, wn);  // the other tile's readers passed the previous barrier
      if (ch + 2 < nch) wn = wload(k0 + 64);
    }
    __syncthreads();
  }
  float* stage = dg_stage + wv * (16 * MS) * CI;
  stage_acc<MS, NS>(stage, acc, quad, col);
  __syncthreads();
  dgrad_epilogue<MS, NS>(stage, lane, [&](int m, int xl) -> long long {
    const long long v = vbase + m * 16 + xl;
    return v < g.mi ? v : -1;
  }, add, mask, da, dzp);
}

// ---------------------------------------------------------------------------
// data gradient of a stride-2 layer by parity class
// ---------------------------------------------------------------------------
// Input voxel q is read by output voxel p = (q + 1 - k) / 2 only through the
// taps with q + 1 - k even: k = 1 where q is even and k in {0, 2} where q is
// odd, per axis.  A wave takes 16 voxels of one x parity in a row
// (x = 2 (i0 + l) + px) and MS rows of one y parity (y = y0 + 2 m) at one z,
// so its tap set (1 to 8 of the 27 taps) is uniform and K = taps x co.
struct S2Geo {
  int n, d, h, w;      // layer input extent
  int od, oh, ow, co;  // layer output extent, output channels
  int nxt, nyg;        // 16-voxel tiles per x parity, y groups (both parities)
  long long nwaves;
};

template <int CI>
__global__ __launch_bounds__(256) void k_conv_bwd_data_s2(const uint16_t* __restrict__ dz,
                                                          const uint16_t* __restrict__ wf, S2Geo g,
                                                          const uint16_t* __restrict__ add,
                                                          const uint16_t* __restrict__ mask,
                                                          uint16_t* __restrict__ da, uint16_t* __restrict__ dzp) {
  constexpr int NS = CI / 16, MS = 8 / NS;
  __shared__ __attribute__((aligned(16))) float dg_stage[4 * 16 * MS * CI];  // the epilogue's staging
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  // wave index in 32 bits (the host checks nwaves < 2^31); a wave past the
  // last one computes nothing but takes part in the epilogue's barrier
  unsigned t = blockIdx.x * 4u + (unsigned)wv;
  const bool active = t < (unsigned)g.nwaves;
  if (!active) t = 0;
  const int ixt = (int)(t % (unsigned)g.nxt);
  t /= (unsigned)g.nxt;
  const int px = (int)(t & 1u);
  t >>= 1;
  const int yg = (int)(t % (unsigned)g.nyg);
  t /= (unsigned)g.nyg;
  const int qz = (int)(t % (unsigned)g.d);
  const int n = (int)(t / (unsigned)g.d);
  const int py = yg & 1, y0 = (yg >> 1) * (2 * MS) + py, i0 = ixt * 16;
  const int pz_odd = qz & 1;
  // taps per axis: 2 on an odd coordinate, 1 on an even one (log2: the parity)
  const int K = active ? g.co << (px + py + pz_odd) : 0, osh = ilog2(g.co);
  const int qx = 2 * (i0 + col) + px;  // this lane's A row
  v4f acc[MS][NS];
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[m][s] = (v4f){0.f, 0.f, 0.f, 0.f};
  const v8bf zero = {};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int k = k0 + 8 * quad;
    const bool kin = k < K;
    const int ti = kin ? (k >> osh) : 0, o = k - (ti << osh);
    const int tx = ti & px, ty = (ti >> px) & py, tz = ti >> (px + py);
    const int kx = px ? 2 * tx : 1, ky = py ? 2 * ty : 1, kz = pz_odd ? 2 * tz : 1;
    const int tap = (kz * 3 + ky) * 3 + kx;
    const int pz = (qz + 1 - kz) >> 1, ppx = (qx + 1 - kx) >> 1;
    const bool okx = kin && qx < g.w && ppx >= 0 && ppx < g.ow && pz >= 0 && pz < g.od;
    const int vrow = ((n * g.od + pz) * g.oh) * g.ow + ppx;  // voxel index of row ppy = 0 (< 2^31)
    v8bf a[MS], b[NS];
#pragma unroll
    for (int m = 0; m < MS; ++m) {
      const int qy = y0 + 2 * m, ppy = (qy + 1 - ky) >> 1;
      const bool v = okx && qy < g.h && ppy >= 0 && ppy < g.oh;
      a[m] = v ? ld8(dz + (long long)(vrow + ppy * g.ow) * g.co + o) : zero;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
      b[s] = kin ? ld8(wf + ((long long)(s * 16 + col) * 27 + (26 - tap)) * g.co + o) : zero;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int m = 0; m < MS; ++m) acc[m][s] = mfma32(a[m], b[s], acc[m][s]);
  }
  // lane holds D[4 quad + r][col]: voxel i0 + 4 quad + r of row m, channel s*16 + col
  float* stage = dg_stage + wv * (16 * MS) * CI;
  stage_acc<MS, NS>(stage, acc, quad, col);
  __syncthreads();
  dgrad_epilogue<MS, NS>(stage, lane, [&](int m, int xl) -> long long {
    const int qy = y0 + 2 * m, qxx = 2 * (i0 + xl) + px;
    if (!active || qy >= g.h || qxx >= g.w) return -1;
    return (((long long)n * g.d + qz) * g.h + qy) * g.w + qxx;
  }, add, mask, da, dzp);
}

// ---------------------------------------------------------------------------
// weight gradient: block (chunk, tap) sums dz[v, o] X[src(v, tap), c] over
// its voxel chunk; partial[chunk][tap][o][c]; db partials from tap 0 blocks
// ---------------------------------------------------------------------------
constexpr int kAllTapsMaxTiles = 2;  // larger (co, ci) take one tap per block
constexpr int WV = 64;       // voxels per LDS tile
constexpr int WP = WV + 8;   // padded LDS row (bf16 elements)

// Transposed LDS store of a 64-voxel tile, two voxels per 32-bit word: lane
// v holds channels c4..c4+3 of voxel v; lanes 2i and 2i+1 swap halves (DPP)
// so that the even lane writes channels c4 and c4+2, the odd lane c4+1 and
// c4+3, each as (voxel 2i, voxel 2i+1).  t[c * WP + v] in bf16 elements.
__device__ __forceinline__ void pair_store4(uint16_t* t, int c4, int lane, v4s val) {
  const uint32_t d0 = (uint32_t)(uint16_t)val[0] | ((uint32_t)(uint16_t)val[1] << 16);
  const uint32_t d1 = (uint32_t)(uint16_t)val[2] | ((uint32_t)(uint16_t)val[3] << 16);
  // quad_perm(1, 0, 3, 2): the value of lane ^ 1
  const uint32_t e0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d0, 0xB1, 0xF, 0xF, false);
  const uint32_t e1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d1, 0xB1, 0xF, 0xF, false);
  const bool odd = lane & 1;
  const uint32_t w0 = odd ? ((e0 >> 16) | (d0 & 0xFFFF0000u)) : ((d0 & 0xFFFFu) | (e0 << 16));
  const uint32_t w1 = odd ? ((e1 >> 16) | (d1 & 0xFFFF0000u)) : ((d1 & 0xFFFFu) | (e1 << 16));
  const int c = c4 + (odd ? 1 : 0);
  uint32_t* t32 = (uint32_t*)t;
  t32[c * (WP / 2) + (lane >> 1)] = w0;
  t32[(c + 2) * (WP / 2) + (lane >> 1)] = w1;
}

// Each wave takes one 16-voxel slice of every 64-voxel tile for all
// (CO/16) x (CI/16) output tiles; the four waves' sums are added through LDS
// at the end.  Tap-0 blocks also sum dz (the bias gradient) with an MFMA
// against a ones operand.
template <int CO, int CI, int S, int U>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dz,
                                                    Geo g, long long vchunk, float* __restrict__ part,
                                                    float* __restrict__ dbpart) {
  constexpr int NO = CO / 16, NC = CI / 16, NTL = NO * NC;
  __shared__ __attribute__((aligned(16))) uint16_t dzT[CO * WP];
  __shared__ __attribute__((aligned(16))) uint16_t xT[CI * WP];
  __shared__ float red[3 * (NTL + NO) * 256];
  const int chunk = blockIdx.x, tap = blockIdx.y;
  const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const long long v0 = (long long)chunk * vchunk;
  const long long v1 = v0 + vchunk < g.mo ? v0 + vchunk : g.mo;
  v4f acc[NTL], accb[NO];
#pragma unroll
  for (int t = 0; t < NTL; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < NO; ++t) accb[t] = (v4f){0.f, 0.f, 0.f, 0.f};
  const short one = 0x3F80;  // bf16 1.0
  const v4s ones = {one, one, one, one};
  const int DU = g.d * U, HU = g.h * U, WU = g.w * U;
  // lane = voxel of the tile; the waves split the channel groups (channels
  // wv*4 + 16 i).  The next tile's dz values and gathered input are loaded
  // while the current tile multiplies.
  v4s dzv[CO / 16], xg[CI / 16];
  auto fetch = [&](long long vt) {
    const long long vv0 = vt + lane;
    const bool vok = vv0 < v1;
#pragma unroll
    for (int i = 0; i < CO / 16; ++i) dzv[i] = vok ? ld4(dz + vv0 * CO + wv * 4 + 16 * i) : (v4s){0, 0, 0, 0};
    long long v = vok ? vv0 : v0;
    const int px = (int)(v % g.ow);
    v /= g.ow;
    const int py = (int)(v % g.oh);
    v /= g.oh;
    const int pz = (int)(v % g.od);
    const int n = (int)(v / g.od);
    const int qz = pz * S + kz - 1, qy = py * S + ky - 1, qx = px * S + kx - 1;
    const bool in = vok && qz >= 0 && qz < DU && qy >= 0 && qy < HU && qx >= 0 && qx < WU;
    const uint16_t* src = x + ((((long long)n * g.d + (in ? qz / U : 0)) * g.h + (in ? qy / U : 0)) * g.w +
                               (in ? qx / U : 0)) * CI;
#pragma unroll
    for (int i = 0; i < CI / 16; ++i) xg[i] = in ? ld4(src + wv * 4 + 16 * i) : (v4s){0, 0, 0, 0};
  };
  if (v0 < v1) fetch(v0);
  for (long long vt = v0; vt < v1; vt += WV) {
    __syncthreads();
    // dz tile and the gathered input of this tap, transposed: dzT[o][voxel], xT[c][voxel]
#pragma unroll
    for (int i = 0; i < CO / 16; ++i) pair_store4(dzT, wv * 4 + 16 * i, lane, dzv[i]);
#pragma unroll
    for (int i = 0; i < CI / 16; ++i) pair_store4(xT, wv * 4 + 16 * i, lane, xg[i]);
    if (vt + WV < v1) fetch(vt + WV);
    __syncthreads();
    const int kofs = wv * 16 + 4 * quad;  // this wave's voxel slice
    v4s a[NO], b[NC];
#pragma unroll
    for (int t = 0; t < NO; ++t) a[t] = *(const v4s*)&dzT[(t * 16 + col) * WP + kofs];
#pragma unroll
    for (int t = 0; t < NC; ++t) b[t] = *(const v4s*)&xT[(t * 16 + col) * WP + kofs];
#pragma unroll
    for (int ot = 0; ot < NO; ++ot)
#pragma unroll
      for (int ct = 0; ct < NC; ++ct) acc[ot * NC + ct] = mfma(a[ot], b[ct], acc[ot * NC + ct]);
    if (tap == 0)
#pragma unroll
      for (int ot = 0; ot < NO; ++ot) accb[ot] = mfma(a[ot], ones, accb[ot]);
  }
  // add the four waves' sums: waves 1..3 park theirs in LDS
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[((wv - 1) * (NTL + NO) + t) * 256 + r * 64 + lane] = acc[t][r];
#pragma unroll
    for (int t = 0; t < NO; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[((wv - 1) * (NTL + NO) + NTL + t) * 256 + r * 64 + lane] = accb[t][r];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[t][r] += red[(k * (NTL + NO) + t) * 256 + r * 64 + lane];
#pragma unroll
    for (int t = 0; t < NO; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) accb[t][r] += red[(k * (NTL + NO) + NTL + t) * 256 + r * 64 + lane];
  }
  // lane holds D[4 quad + r][col]: o = ot*16 + 4 quad + r, c = ct*16 + col
#pragma unroll
  for (int ot = 0; ot < NO; ++ot)
#pragma unroll
    for (int ct = 0; ct < NC; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = ot * 16 + 4 * quad + r, c = ct * 16 + col;
        part[(((long long)chunk * 27 + tap) * CO + o) * CI + c] = acc[ot * NC + ct][r];
      }
  if (tap == 0 && col == 0)  // every column of the ones product holds the row sum
#pragma unroll
    for (int ot = 0; ot < NO; ++ot)
#pragma unroll
      for (int r = 0; r < 4; ++r) dbpart[(long long)chunk * CO + ot * 16 + 4 * quad + r] = accb[ot][r];
}

// Weight gradient for small channel counts ((CO/16) (CI/16) <= 2): a block
// owns a voxel chunk and all 27 taps, so its dz tile is staged once; wave w
// takes taps w, w + 4, ... (whole 64-voxel tiles), so no cross-wave sums are
// needed.  Partials as in k_conv_bwd_w (grid.y = 1, tap index inside).
template <int CO, int CI, int S, int U>
__global__ __launch_bounds__(256) void k_conv_bwd_w_taps(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ dz, Geo g, long long vchunk,
                                                         float* __restrict__ part, float* __restrict__ dbpart) {
  constexpr int NO = CO / 16, NC = CI / 16, NTL = NO * NC, SLOTS = 7;  // ceil(27 / 4)
  __shared__ __attribute__((aligned(16))) uint16_t dzT[CO * WP];
  __shared__ __attribute__((aligned(16))) uint16_t xT[4][CI * WP];
  const int chunk = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const long long v0 = (long long)chunk * vchunk;
  const long long v1 = v0 + vchunk < g.mo ? v0 + vchunk : g.mo;
  v4f acc[SLOTS][NTL], accb[NO];
#pragma unroll
  for (int t = 0; t < SLOTS; ++t)
#pragma unroll
    for (int i = 0; i < NTL; ++i) acc[t][i] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < NO; ++t) accb[t] = (v4f){0.f, 0.f, 0.f, 0.f};
  const short one = 0x3F80;  // bf16 1.0
  const v4s ones = {one, one, one, one};
  const int DU = g.d * U, HU = g.h * U, WU = g.w * U;
  uint16_t* myx = xT[wv];
  for (long long vt = v0; vt < v1; vt += WV) {
    __syncthreads();
    for (int i = threadIdx.x; i < WV * (CO / 4); i += 256) {
      const int vl = i / (CO / 4), c4 = (i % (CO / 4)) * 4;
      const long long v = vt + vl;
      v4s val = {0, 0, 0, 0};
      if (v < v1) val = ld4(dz + v * CO + c4);
#pragma unroll
      for (int j = 0; j < 4; ++j) dzT[(c4 + j) * WP + vl] = (uint16_t)val[j];
    }
    // this lane's voxel decomposition for the gathers (lane = voxel of the tile)
    long long vv = vt + lane;
    const bool vok = vv < v1;
    if (!vok) vv = v0;
    const int px = (int)(vv % g.ow);
    vv /= g.ow;
    const int py = (int)(vv % g.oh);
    vv /= g.oh;
    const int pz = (int)(vv % g.od);
    const int n = (int)(vv / g.od);
    // this lane's voxel of the input shifted by a tap; the next slot's gather
    // is in flight while the current slot multiplies
    v4s xv[CI / 4];
    auto gather = [&](int tap) {
      if (tap >= 27) return;
      const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
      const int qz = pz * S + kz - 1, qy = py * S + ky - 1, qx = px * S + kx - 1;
      const bool in = vok && qz >= 0 && qz < DU && qy >= 0 && qy < HU && qx >= 0 && qx < WU;
      const uint16_t* src = x + ((((long long)n * g.d + (in ? qz / U : 0)) * g.h + (in ? qy / U : 0)) * g.w +
                                 (in ? qx / U : 0)) * CI;
#pragma unroll
      for (int c4 = 0; c4 < CI; c4 += 4) xv[c4 / 4] = in ? ld4(src + c4) : (v4s){0, 0, 0, 0};
    };
    gather(wv);
#pragma unroll
    for (int slot = 0; slot < SLOTS; ++slot) {
      const int tap = wv + 4 * slot;
      __syncthreads();  // dzT ready (slot 0) / previous slot's reads done
      if (tap < 27)
#pragma unroll
        for (int c4 = 0; c4 < CI; c4 += 4)
#pragma unroll
          for (int j = 0; j < 4; ++j) myx[(c4 + j) * WP + lane] = (uint16_t)xv[c4 / 4][j];
      gather(tap + 4);
      __syncthreads();
      if (tap < 27) {
#pragma unroll
        for (int kk = 0; kk < WV / 16; ++kk) {
          const int kofs = kk * 16 + 4 * quad;
          v4s a[NO], b[NC];
#pragma unroll
          for (int t = 0; t < NO; ++t) a[t] = *(const v4s*)&dzT[(t * 16 + col) * WP + kofs];
#pragma unroll
          for (int t = 0; t < NC; ++t) b[t] = *(const v4s*)&myx[(t * 16 + col) * WP + kofs];
#pragma unroll
          for (int ot = 0; ot < NO; ++ot)
#pragma unroll
            for (int ct = 0; ct < NC; ++ct) acc[slot][ot * NC + ct] = mfma(a[ot], b[ct], acc[slot][ot * NC + ct]);
          if (slot == 0 && wv == 0)
#pragma unroll
            for (int ot = 0; ot < NO; ++ot) accb[ot] = mfma(a[ot], ones, accb[ot]);
        }
      }
    }
  }
#pragma unroll
  for (int slot = 0; slot < SLOTS; ++slot) {
    const int tap = wv + 4 * slot;
    if (tap >= 27) break;
#pragma unroll
    for (int ot = 0; ot < NO; ++ot)
#pragma unroll
      for (int ct = 0; ct < NC; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = ot * 16 + 4 * quad + r, c = ct * 16 + col;
          part[(((long long)chunk * 27 + tap) * CO + o) * CI + c] = acc[slot][ot * NC + ct][r];
        }
  }
  if (wv == 0 && col == 0)
#pragma unroll
    for (int ot = 0; ot < NO; ++ot)
#pragma unroll
      for (int r = 0; r < 4; ++r) dbpart[(long long)chunk * CO + ot * 16 + 4 * quad + r] = accb[ot][r];
}

// dw[o][k][c] = sum over chunks of part[chunk][k][o][c] (and db likewise):
// a block takes 64 consecutive outputs, its four waves every fourth chunk,
// and the four partial sums are added in wave order (deterministic)
__global__ __launch_bounds__(256) void k_bwd_w_reduce(const float* __restrict__ part,
                                                      const float* __restrict__ dbpart, int nchunk, int co, int ci,
                                                      float* __restrict__ dw, float* __restrict__ db) {
  // 16 outputs per block, the chunks split over 16 groups of lanes (group g
  // sums chunks g, g + 16, ... in order), the 16 group sums added in group
  // order: a fixed summation order, so the result is deterministic.  The
  // blocks past the weights' sum the bias partials.
  __shared__ float sh[16][17];
  const int e = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int n = 27 * co * ci;
  const int nb = (n + 15) / 16;
  const bool bias = (int)blockIdx.x >= nb;
  const int i = (bias ? (int)blockIdx.x - nb : (int)blockIdx.x) * 16 + e;
  const int lim = bias ? co : n;
  const float* src = bias ? dbpart : part;
  const long long stride = bias ? co : n;
  float s = 0.0f;
  if (i < lim) {
#pragma unroll 4
    for (int k = grp; k < nchunk; k += 16) s += src[(long long)k * stride + i];
  }
  sh[grp][e] = s;
  __syncthreads();
  if (grp != 0 || i >= lim) return;
  float t = 0.0f;
#pragma unroll
  for (int g = 0; g < 16; ++g) t += sh[g][e];
  if (bias) {
    db[i] = t;
  } else {
    const int c = i % ci, o = (i / ci) % co, tap = i / (ci * co);
    dw[((long long)o * 27 + tap) * ci + c] = t;
  }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// wu[c][a][o] (a = (az * 4 + ay) * 4 + ax) = sum over k in F(az) x F(ay) x F(ax)
// of w[o][k][c], summed in FP32 in tap order and rounded once to bf16
__global__ void k_fold_up_w(const uint16_t* __restrict__ w, int co, int ci, uint16_t* __restrict__ wu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over [c][a][o]
  if (i >= ci * 64 * co) return;
  const int o = i % co, a = (i / co) % 64, c = i / (co * 64);
  const int az = a >> 4, ay = (a >> 2) & 3, ax = a & 3;
  float sum = 0.0f;
  for (int kz = max(0, 2 - az); kz <= min(2, 3 - az); ++kz)
    for (int ky = max(0, 2 - ay); ky <= min(2, 3 - ay); ++ky)
      for (int kx = max(0, 2 - ax); kx <= min(2, 3 - ax); ++kx)
        sum += bf2f(w[((long long)o * 27 + (kz * 3 + ky) * 3 + kx) * ci + c]);
  wu[i] = f2bf(sum);
}

__global__ void k_flip_w(const uint16_t* __restrict__ w, int co, int ci, uint16_t* __restrict__ wf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over [o][k][c]
  if (i >= co * 27 * ci) return;
  const int c = i % ci, k = (i / ci) % 27, o = i / (ci * 27);
  wf[((long long)c * 27 + (26 - k)) * co + o] = w[i];
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long count, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, uint16_t* __restrict__ pb) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

__global__ void k_normalize(const float* __restrict__ x, int c, long long vox, long long total,
                            const float* __restrict__ shift, const float* __restrict__ scale, float* xn) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int ch = (int)((i / vox) % c);
  xn[i] = (x[i] - shift[ch]) * scale[ch];
}

// one thread per voxel: its c channels (coalesced over voxels per channel),
// written as cpad bf16 with 16-byte stores
__global__ void k_pack(const float* __restrict__ xn, int c, long long vox, int cpad, long long nvox,
                       uint16_t* __restrict__ xb) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // over [n][vox]
  if (q >= nvox) return;
  const long long n = q / vox, v = q - n * vox;
  for (int c0 = 0; c0 < cpad; c0 += 8) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ch = c0 + 2 * j;
      const uint32_t lo = ch < c ? f2bf(xn[(n * c + ch) * vox + v]) : 0u;
      const uint32_t hi = ch + 1 < c ? f2bf(xn[(n * c + ch + 1) * vox + v]) : 0u;
      w[j] = lo | (hi << 16);
    }
    *(uint4*)(xb + q * cpad + c0) = (uint4){w[0], w[1], w[2], w[3]};
  }
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
  __syncthreads();
  return s;
}

constexpr int kLossBlocks = 1024;
constexpr int kLossMaxSamples = 1024;  // mass term: per-sample sums follow the partials in ws

// per-sample sums of the phase-field residual d = xn + rs r - tn (channel 0),
// FP64: blockIdx.y = sample, blockIdx.x = one of np partial ranges, then
// k_mass_final adds the np partials of each sample in a fixed order
__global__ __launch_bounds__(256) void k_mass_residual(const float* __restrict__ xn, const float* __restrict__ tn,
                                                       const uint16_t* __restrict__ r,
                                                       const float* __restrict__ rs, int c, long long vox,
                                                       int cpad, int np, double* __restrict__ mpart) {
  __shared__ double sh[4];
  const long long n = blockIdx.y;
  const float sc = rs ? rs[0] : 1.0f;
  double s = 0.0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < vox; v += (long long)np * blockDim.x) {
    const long long j = n * c * vox + v;
    s += (double)(xn[j] + sc * bf2f(r[(n * vox + v) * cpad]) - tn[j]);
  }
  const double b = block_sum(s, sh);
  if (threadIdx.x == 0) mpart[n * np + blockIdx.x] = b;
}

__global__ void k_mass_final(const double* __restrict__ mpart, int n, int np, double* __restrict__ msum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < np; ++k) s += mpart[(long long)i * np + k];
  msum[i] = s;
}

// one thread per voxel (grid-stride): its cpad residual channels read and
// its gradient written with 16-byte accesses, the c real channels' d^2
// accumulated in FP64; per-block partials in a fixed order
__global__ __launch_bounds__(256) void k_residual_loss(const float* __restrict__ xn, const float* __restrict__ tn,
                                                       const uint16_t* __restrict__ r,
                                                       const float* __restrict__ rs, int c, long long vox,
                                                       int cpad, long long nvox, float inv_count,
                                                       const double* __restrict__ msum, float mgrad,
                                                       uint16_t* __restrict__ dr, double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nvox;
       q += (long long)gridDim.x * blockDim.x) {  // over [n][vox]
    const long long n = q / vox, v = q - n * vox;
    const float mg = msum ? mgrad * (float)msum[n] : 0.0f;  // d/dd of the mass term (channel 0)
    for (int c0 = 0; c0 < cpad; c0 += 8) {
      const uint4 rv = *(const uint4*)(r + q * cpad + c0);
      const uint32_t rw[4] = {rv.x, rv.y, rv.z, rv.w};
      uint32_t gw[4];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int ch = c0 + j;
        float gval = 0.0f;
        if (ch < c) {
          const long long jx = (n * c + ch) * vox + v;
          const float sc = rs ? rs[ch] : 1.0f;
          const float d = xn[jx] + sc * bf2f((uint16_t)(rw[j >> 1] >> (16 * (j & 1)))) - tn[jx];
          s += (double)d * d;
          float gd = 2.0f * d * inv_count;
          if (ch == 0) gd += mg;
          gval = sc * gd;
        }
        const uint32_t b = f2bf(gval);
        if (j & 1) gw[j >> 1] |= b << 16;
        else gw[j >> 1] = b;
      }
      *(uint4*)(dr + q * cpad + c0) = (uint4){gw[0], gw[1], gw[2], gw[3]};
    }
  }
  const double b = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// loss = scale * sum(part) + mw * sum_n (msum[n] / vox)^2 / n (mass term, if msum)
__global__ void k_sum_parts(const double* __restrict__ part, int np, double scale, const double* __restrict__ msum,
                            int n, double vox, double mw, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += part[i];
    s *= scale;
    if (msum) {
      double m = 0.0;
      for (int i = 0; i < n; ++i) m += (msum[i] / vox) * (msum[i] / vox);
      s += mw * m / n;
    }
    *out = s;
  }
}

__global__ void k_unpack(const float* __restrict__ xn, const uint16_t* __restrict__ r, const float* __restrict__ rs,
                         int c, long long vox, int cpad, long long total, const float* __restrict__ shift,
                         const float* __restrict__ scale, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // over [n][c][vox]
  if (i >= total) return;
  const long long v = i % vox;
  const int ch = (int)((i / vox) % c);
  const long long n = i / (vox * c);
  const float sc = rs ? rs[ch] : 1.0f;
  out[i] = (xn[i] + sc * bf2f(r[(n * vox + v) * cpad + ch])) / scale[ch] + shift[ch];
}

__global__ void k_coarsen(const float* __restrict__ phi, const float* __restrict__ u, const float* __restrict__ p,
                          int nx, int ny, int nz, int z0c, int dw, float* __restrict__ out) {
  const int hx = nx / 2, hy = ny / 2;
  const long long plane = (long long)hx * hy, vol = plane * dw;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // over [5][dw][hy][hx]
  if (i >= 5 * vol) return;
  const int ch = (int)(i / vol);
  const long long r = i % vol;
  const int zc = (int)(r / plane) + z0c, yc = (int)((r % plane) / hx), xc = (int)(r % hx);
  float s = 0.0f;
  if (2 * zc + 1 < nz) {
    const long long N = (long long)nx * ny * nz;
    const float* f = ch == 0 ? phi : (ch == 4 ? p : u + (long long)(ch - 1) * N);
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          s += f[((long long)(2 * zc + dz) * ny + (2 * yc + dy)) * nx + (2 * xc + dx)];
    s *= 0.125f;
  }
  out[i] = s;
}

__global__ __launch_bounds__(256) void k_phi_budget(const float* __restrict__ x, int c, int d, int h, int w,
                                                    double* __restrict__ sums) {
  __shared__ double sh[4];
  const int n = blockIdx.x;
  const long long plane = (long long)h * w, vox = plane * d;
  const float* phi = x + (long long)n * c * vox;
  const float* uz = phi + 3 * vox;
  double s = 0.0, fi = 0.0, fo = 0.0;
  for (long long i = threadIdx.x; i < vox; i += blockDim.x) s += phi[i];
  for (long long i = threadIdx.x; i < plane; i += blockDim.x) {
    fi += (double)phi[i] * uz[i];
    fo += (double)phi[(d - 1) * plane + i] * uz[(d - 1) * plane + i];
  }
  const double a = block_sum(s, sh);
  const double b = block_sum(fi, sh);
  const double e = block_sum(fo, sh);
  if (threadIdx.x == 0) {
    sums[3 * n + 0] = a;
    sums[3 * n + 1] = b;
    sums[3 * n + 2] = e;
  }
}

__global__ void k_gather(const float* __restrict__ store, long long rows, long long len,
                         const long long* __restrict__ idx, int n, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // over [n][len]
  if (i >= (long long)n * len) return;
  const long long j = i / len, e = i % len;
  const long long r = idx[j];
  out[i] = (r >= 0 && r < rows) ? store[r * len + e] : __int_as_float(0x7fc00000);
}

bool chan_ok(int c) { return c == 16 || c == 32 || c == 64; }

unsigned blocks_for(long long n, int b) { return (unsigned)((n + b - 1) / b); }

template <int CO, int S, int U>
void launch_fwd(const Geo& g, const uint16_t* x, const uint16_t* w, const float* b, const uint16_t* skip,
                uint16_t* y, uint16_t* yr, int relu, hipStream_t st) {
  constexpr int MS = 8 / (CO / 16);
  const long long per_block = 4LL * 16 * MS;
  hipLaunchKernelGGL((k_conv_fwd<CO, S, U>), dim3(blocks_for(g.mo, (int)per_block)), dim3(256), 0, st, x, w, b,
                     skip, y, yr, g, relu);
}

template <int S, int U>
void launch_fwd_su(const Geo& g, const uint16_t* x, const uint16_t* w, const float* b, const uint16_t* skip,
                   uint16_t* y, uint16_t* yr, int relu, hipStream_t st) {
  if (g.co == 16) launch_fwd<16, S, U>(g, x, w, b, skip, y, yr, relu, st);
  else if (g.co == 32) launch_fwd<32, S, U>(g, x, w, b, skip, y, yr, relu, st);
  else launch_fwd<64, S, U>(g, x, w, b, skip, y, yr, relu, st);
}

template <int CI, int S, int U>
void launch_bwd_data(const Geo& g, const uint16_t* dz, const uint16_t* wt, const uint16_t* add,
                     const uint16_t* mask, uint16_t* da, uint16_t* dzp, hipStream_t st) {
  constexpr int MS = 8 / (CI / 16);
  const long long per_block = 4LL * 16 * MS;
  hipLaunchKernelGGL((k_conv_bwd_data<CI, S, U>), dim3(blocks_for(g.mi, (int)per_block)), dim3(256), 0, st, dz,
                     wt, g, add, mask, da, dzp);
}

template <int CI>
void launch_bwd_data_up2(const Geo& g, const uint16_t* dz, const uint16_t* wu, const uint16_t* add,
                         const uint16_t* mask, uint16_t* da, uint16_t* dzp, hipStream_t st) {
  constexpr int MS = 8 / (CI / 16);
  const long long per_block = 4LL * 16 * MS;
  hipLaunchKernelGGL((k_conv_bwd_data_up2<CI>), dim3(blocks_for(g.mi, (int)per_block)), dim3(256), 0, st, dz, wu,
                     g, add, mask, da, dzp);
}

template <int S, int U>
void launch_bwd_data_su(const Geo& g, const uint16_t* dz, const uint16_t* wt, const uint16_t* add,
                        const uint16_t* mask, uint16_t* da, uint16_t* dzp, hipStream_t st) {
  if (g.ci == 16) launch_bwd_data<16, S, U>(g, dz, wt, add, mask, da, dzp, st);
  else if (g.ci == 32) launch_bwd_data<32, S, U>(g, dz, wt, add, mask, da, dzp, st);
  else launch_bwd_data<64, S, U>(g, dz, wt, add, mask, da, dzp, st);
}

template <int CI>
void launch_bwd_data_s2(const Geo& g, const uint16_t* dz, const uint16_t* wf, const uint16_t* add,
                        const uint16_t* mask, uint16_t* da, uint16_t* dzp, hipStream_t st) {
  constexpr int MS = 8 / (CI / 16);
  S2Geo s2;
  s2.n = g.n;
  s2.d = g.d;
  s2.h = g.h;
  s2.w = g.w;
  s2.od = g.od;
  s2.oh = g.oh;
  s2.ow = g.ow;
  s2.co = g.co;
  s2.nxt = ((g.w + 1) / 2 + 15) / 16;
  s2.nyg = 2 * (((g.h + 1) / 2 + MS - 1) / MS);
  s2.nwaves = (long long)s2.nxt * 2 * s2.nyg * g.d * g.n;  // < 2^31: checked by sg_conv3d_bwd_data
  hipLaunchKernelGGL((k_conv_bwd_data_s2<CI>), dim3(blocks_for(s2.nwaves, 4)), dim3(256), 0, st, dz, wf, s2, add,
                     mask, da, dzp);
}

template <int CO, int CI, int S, int U>
void launch_bwd_w_one(const Geo& g, const uint16_t* x, const uint16_t* dz, int nchunk, long long vchunk,
                      float* part, float* dbpart, hipStream_t st) {
  if constexpr ((CO / 16) * (CI / 16) <= kAllTapsMaxTiles)  // all taps per block
    hipLaunchKernelGGL((k_conv_bwd_w_taps<CO, CI, S, U>), dim3(nchunk), dim3(256), 0, st, x, dz, g, vchunk, part,
                       dbpart);
  else
    hipLaunchKernelGGL((k_conv_bwd_w<CO, CI, S, U>), dim3(nchunk, 27), dim3(256), 0, st, x, dz, g, vchunk, part,
                       dbpart);
}

template <int CO, int S, int U>
void launch_bwd_w_co(const Geo& g, const uint16_t* x, const uint16_t* dz, int nchunk, long long vchunk,
                     float* part, float* dbpart, hipStream_t st) {
  if (g.ci == 16) launch_bwd_w_one<CO, 16, S, U>(g, x, dz, nchunk, vchunk, part, dbpart, st);
  else if (g.ci == 32) launch_bwd_w_one<CO, 32, S, U>(g, x, dz, nchunk, vchunk, part, dbpart, st);
  else launch_bwd_w_one<CO, 64, S, U>(g, x, dz, nchunk, vchunk, part, dbpart, st);
}

template <int S, int U>
void launch_bwd_w_su(const Geo& g, const uint16_t* x, const uint16_t* dz, int nchunk, long long vchunk,
                     float* part, float* dbpart, hipStream_t st) {
  if (g.co == 16) launch_bwd_w_co<16, S, U>(g, x, dz, nchunk, vchunk, part, dbpart, st);
  else if (g.co == 32) launch_bwd_w_co<32, S, U>(g, x, dz, nchunk, vchunk, part, dbpart, st);
  else launch_bwd_w_co<64, S, U>(g, x, dz, nchunk, vchunk, part, dbpart, st);
}

template <int CI, int CO, int U, int MODE>
void launch_halo_c(int n, int d, int h, int w, const uint16_t* x, const uint16_t* wgt, const float* bias,
                   const uint16_t* other, const uint16_t* mask, uint16_t* y, uint16_t* y2, int relu, hipStream_t st) {
  using T = HaloTile<CI, CO, U>;
  HGeo g;
  g.n = n;
  g.d = d;
  g.h = h;
  g.w = w;
  g.od = U * d;
  g.oh = U * h;
  g.ow = U * w;
  g.ntx = (g.ow + 15) / 16;
  g.nty = (g.oh + T::TY - 1) / T::TY;
  g.ntz = (g.od + T::TZ - 1) / T::TZ;
  const long long blocks = (long long)g.ntx * g.nty * g.ntz * n;
  hipLaunchKernelGGL((k_conv_halo<CI, CO, U, MODE>), dim3((unsigned)blocks), dim3(256), 0, st, x, wgt, bias, other,
                     mask, y, y2, g, relu);
}

// Every same-size stride-1 layer (forward and data gradient) takes the halo
// tile: at 64 channels a block holds only 8 rows and stages 3.4x its own
// voxels, yet it beats the direct kernel's 27 gathers per voxel (measured
// per layer width).  With upsampling: the decoder's 32 -> 16 and 64 -> 32.
bool halo_fwd(int ci, int co, int stride, int up) {
  if (stride != 1) return false;
  if (up == 1) return ci == co;
  return (ci == 32 && co == 16) || (ci == 64 && co == 32);
}
bool halo_data(int) { return true; }

template <int MODE>
void launch_halo(int n, int d, int h, int w, int c, const uint16_t* x, const uint16_t* wgt, const float* bias,
                 const uint16_t* other, const uint16_t* mask, uint16_t* y, uint16_t* y2, int relu, hipStream_t st) {
  if (c == 16) launch_halo_c<16, 16, 1, MODE>(n, d, h, w, x, wgt, bias, other, mask, y, y2, relu, st);
  else if (c == 32) launch_halo_c<32, 32, 1, MODE>(n, d, h, w, x, wgt, bias, other, mask, y, y2, relu, st);
  else launch_halo_c<64, 64, 1, MODE>(n, d, h, w, x, wgt, bias, other, mask, y, y2, relu, st);
}

// ---------------------------------------------------------------------------
// weight gradient of stride-1 layers from LDS halo bricks
// ---------------------------------------------------------------------------
// A block walks output bricks of TZ x TY rows of 16 voxels.  Per brick it
// stages dz transposed (channel-major, dzT[o][row][x]) and the input with a
// one-voxel halo transposed (xT[c][hz][hy][hx], in upsampled coordinates for
// U = 2), once.  Wave w owns the nine taps with kz = w: per 32-voxel K step
// it reads the dz operand and one new halo row segment (two aligned 16-byte
// reads, from which the three kx shifts are cut with byte alignment), and
// keeps the rows of the three ky taps in registers --
// dW[o][tap][c] += dz[p][o] X[p + tap - 1][c].  Layers are split into slices
// of 16 output channels and at most 32 input channels (blockIdx.y), which
// keeps a wave's accumulators and rows within 256 registers (two waves per
// SIMD).  The per-block sums go to the same partial layout as the direct
// kernels.
template <int CO, int CI>
struct WHalo {
  static_assert(CO == 16 && (CI == 16 || CI == 32), "slices of 16 output and 16 or 32 input channels");
  static constexpr int NO = CO / 16, NC = CI / 16;
  static constexpr int TZ = CI == 16 ? 4 : 2, TY = 8;
  static constexpr int R = TZ * TY;                 // rows of 16 voxels
  static_assert(TZ % 2 == 0, "the K step pairs rows of adjacent z planes");
  static constexpr int HX = 18, HXP = 24, HY = TY + 2, HZ = TZ + 2;
  static_assert(HXP >= 20, "halo rows are staged 20 wide");
  static constexpr int DZS = R * 16 + 8;            // dzT channel stride (elements), 4 banks apart
  static constexpr int XB = HZ * HY * HXP;          // halo elements per channel
  static constexpr int XCS = XB + 2 * ((20 - (XB / 2) % 64 + 64) % 64);  // 20 banks apart
  static constexpr int DZ_ELEMS = CO * DZS, X_ELEMS = CI * XCS;
  // the 16-channel slice has the registers to load the next brick while it
  // multiplies the current one
  static constexpr bool PF = CI == 16;
};
constexpr int kWHaloBlocks = 1024;

struct WGeo {
  int n, d, h, w;     // layer input extent
  int od, oh, ow;     // output extent (= U x input)
  int ntx, nty, ntz;  // bricks along x, y, z
  int nbricks;
};

__device__ __forceinline__ v8bf as_bf8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const uint4 v = {a, b, c, d};
  return __builtin_bit_cast(v8bf, v);
}

template <int CO, int CI, int U, bool PF>
__global__ __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_bwd_w_halo(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ dz, WGeo g, int cot, int cit,
                                                         float* __restrict__ part, float* __restrict__ dbpart) {
  using T = WHalo<CO, CI>;
  constexpr int NO = T::NO, NC = T::NC, TZ = T::TZ, TY = T::TY, R = T::R;
  constexpr int HXP = T::HXP, HY = T::HY, HZ = T::HZ, DZS = T::DZS, XCS = T::XCS;
  __shared__ __attribute__((aligned(16))) uint16_t dzT[T::DZ_ELEMS];
  __shared__ __attribute__((aligned(16))) uint16_t xT[T::X_ELEMS];
  const int lane = threadIdx.x & 63, kz = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const int nci = cit / CI;                                  // channel slices of this block
  const int ci0 = (blockIdx.y % nci) * CI, co0 = (blockIdx.y / nci) * CO;
  v4f acc[9][NO * NC], accb[NO];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < NO * NC; ++i) acc[t][i] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < NO; ++i) accb[i] = (v4f){0.f, 0.f, 0.f, 0.f};
  v8bf ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = (__bf16)1.0f;
  // Staging items: dz items are 4 consecutive x voxels x 8 channels of an
  // output row, x items 4 consecutive halo voxels x 8 channels of a halo row
  // (the halo rows are staged 20 wide, inside HXP).  Every load of a brick
  // is issued before the first is used, into registers; with PF the next
  // brick's loads are in flight while the current brick is multiplied.
  constexpr int DZ_ITEMS = R * 4 * (CO / 8), X_ITEMS = HZ * HY * 5 * (CI / 8);
  constexpr int DZ_PT = (DZ_ITEMS + 191) / 192, X_PT = (X_ITEMS + 191) / 192;
  uint4 vd[DZ_PT][4], vx[X_PT][4];
  auto load = [&](int b) {
    int r0 = b;
    const int tx = r0 % g.ntx;
    r0 /= g.ntx;
    const int ty = r0 % g.nty;
    r0 /= g.nty;
    const int tz = r0 % g.ntz;
    const int n = r0 / g.ntz;
    const int x0 = tx * 16, y0 = ty * TY, z0 = tz * TZ;
#pragma unroll
    for (int k = 0; k < DZ_PT; ++k) {
      const int i = threadIdx.x + 192 * k;
      const int c8 = (i % (CO / 8)) * 8, v4 = (i / (CO / 8)) * 4;
      const int gz = z0 + (v4 >> 4) / TY, gy = y0 + (v4 >> 4) % TY;
      const bool rowok = (DZ_ITEMS % 192 == 0 || i < DZ_ITEMS) && gz < g.od && gy < g.oh;
      const long long row = (((long long)n * g.od + gz) * g.oh + gy) * g.ow;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gx = x0 + (v4 & 15) + e;
        vd[k][e] = (uint4){0u, 0u, 0u, 0u};
        if (rowok && gx < g.ow) vd[k][e] = *(const uint4*)(dz + (row + gx) * cot + co0 + c8);
      }
    }
#pragma unroll
    for (int k = 0; k < X_PT; ++k) {
      const int i = threadIdx.x + 192 * k;
      const int c8 = (i % (CI / 8)) * 8, hv = i / (CI / 8);
      const int hx4 = (hv % 5) * 4, hy = (hv / 5) % HY, hz = hv / (5 * HY);
      const int qy = y0 - 1 + hy, qz = z0 - 1 + hz;
      const bool rowok = (X_ITEMS % 192 == 0 || i < X_ITEMS) && qy >= 0 && qy < g.oh && qz >= 0 && qz < g.od;
      const long long row = (((long long)n * g.d + qz / U) * g.h + qy / U) * g.w;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int qx = x0 - 1 + hx4 + e;
        vx[k][e] = (uint4){0u, 0u, 0u, 0u};
        if (rowok && qx >= 0 && qx < g.ow) vx[k][e] = *(const uint4*)(x + (row + qx / U) * cit + ci0 + c8);
      }
    }
  };
  // transposed LDS writes: channel c8 + j of the item's 4 voxels in one 8-byte
  // write; v_perm pairs the 16-bit halves of two voxels' words
  auto put = [](uint16_t* dst, const uint4 (&v)[4], int j) {
    const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      w[e] = (j >> 1) == 0 ? v[e].x : (j >> 1) == 1 ? v[e].y : (j >> 1) == 2 ? v[e].z : v[e].w;
    *(uint2*)dst = (uint2){__builtin_amdgcn_perm(w[1], w[0], sel), __builtin_amdgcn_perm(w[3], w[2], sel)};
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < DZ_PT; ++k) {
      const int i = threadIdx.x + 192 * k;
      if (DZ_ITEMS % 192 == 0 || i < DZ_ITEMS) {
        const int c8 = (i % (CO / 8)) * 8, v4 = (i / (CO / 8)) * 4;
#pragma unroll
        for (int j = 0; j < 8; ++j) put(&dzT[(c8 + j) * DZS + v4], vd[k], j);
      }
    }
#pragma unroll
    for (int k = 0; k < X_PT; ++k) {
      const int i = threadIdx.x + 192 * k;
      if (X_ITEMS % 192 == 0 || i < X_ITEMS) {
        const int c8 = (i % (CI / 8)) * 8, hv = i / (CI / 8);
        const int hx4 = (hv % 5) * 4, hy = (hv / 5) % HY, hz = hv / (5 * HY);
#pragma unroll
        for (int j = 0; j < 8; ++j) put(&xT[(c8 + j) * XCS + (hz * HY + hy) * HXP + hx4], vx[k], j);
      }
    }
  };
  // brick walk: the blocks of one XCD start on adjacent bricks (xcd_item)
  const int G = gridDim.x;
  const int v0 = xcd_item(blockIdx.x, G);
  if (PF && v0 < g.nbricks) load(v0);
  for (int b = v0; b < g.nbricks; b += G) {
    if (!PF) load(b);
    __syncthreads();  // the previous brick's reads are done
    store();
    __syncthreads();
    if (PF && b + G < g.nbricks) load(b + G);
    // K step of 32 voxels: quads 0-1 hold x 0..15 of row (2 zp, ry), quads
    // 2-3 those of row (2 zp + 1, ry).  The halo row a lane reads for tap
    // (kz, ky) is (2 zp + quad / 2 + kz, ry + ky), so walking ry keeps the
    // three rows of the ky taps in registers (with their kx shifts cut
    // once) and reads one new halo row per step.
    const int xo = 8 * (quad & 1);
#pragma unroll
    for (int zp = 0; zp < TZ / 2; ++zp) {
      const int rz = 2 * zp + (quad >> 1);
      v8bf win[3][NC][3];  // [row slot][ct][kx]
      auto ld_row = [&](int hy, v8bf (&w)[NC][3]) {
#pragma unroll
        for (int ct = 0; ct < NC; ++ct) {
          const uint16_t* src = &xT[(ct * 16 + col) * XCS + ((rz + kz) * HY + hy) * HXP + xo];
          const uint4 lo = *(const uint4*)src, hi = *(const uint4*)(src + 8);
          // window elements kx .. kx + 7 of the 16 read: kx = 1 shifts by one bf16
          w[ct][0] = as_bf8(lo.x, lo.y, lo.z, lo.w);
          w[ct][1] = as_bf8(__builtin_amdgcn_alignbyte(lo.y, lo.x, 2), __builtin_amdgcn_alignbyte(lo.z, lo.y, 2),
                            __builtin_amdgcn_alignbyte(lo.w, lo.z, 2), __builtin_amdgcn_alignbyte(hi.x, lo.w, 2));
          w[ct][2] = as_bf8(lo.y, lo.z, lo.w, hi.x);
        }
      };
      ld_row(0, win[0]);
      ld_row(1, win[1]);
#pragma unroll
      for (int ry = 0; ry < TY; ++ry) {
        ld_row(ry + 2, win[(ry + 2) % 3]);
        v8bf a[NO];
#pragma unroll
        for (int ot = 0; ot < NO; ++ot) a[ot] = *(const v8bf*)&dzT[(ot * 16 + col) * DZS + (rz * TY + ry) * 16 + xo];
        if (kz == 0)
#pragma unroll
          for (int ot = 0; ot < NO; ++ot) accb[ot] = mfma32(a[ot], ones, accb[ot]);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
          for (int ct = 0; ct < NC; ++ct)
#pragma unroll
            for (int ot = 0; ot < NO; ++ot)
#pragma unroll
              for (int kx = 0; kx < 3; ++kx)
                acc[ky * 3 + kx][ot * NC + ct] = mfma32(a[ot], win[(ry + ky) % 3][ct][kx], acc[ky * 3 + kx][ot * NC + ct]);
      }
    }
  }
  // lane holds D[4 quad + r][col]: o = ot*16 + 4 quad + r, c = ct*16 + col
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int tap = kz * 9 + t;
#pragma unroll
    for (int ot = 0; ot < NO; ++ot)
#pragma unroll
      for (int ct = 0; ct < NC; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[(((long long)blockIdx.x * 27 + tap) * cot + co0 + ot * 16 + 4 * quad + r) * cit + ci0 + ct * 16 +
               col] = acc[t][ot * NC + ct][r];
  }
  if (kz == 0 && col == 0 && ci0 == 0)
#pragma unroll
    for (int ot = 0; ot < NO; ++ot)
#pragma unroll
      for (int r = 0; r < 4; ++r) dbpart[(long long)blockIdx.x * cot + co0 + ot * 16 + 4 * quad + r] = accb[ot][r];
}

// voxel chunking of the weight gradient: about 2048 blocks (the per-tap
// kernel has 27 blocks per chunk, the all-taps kernel one)
// the halo-brick weight gradient takes every stride-1 layer (in slices of 16
// output and at most 32 input channels)
bool whalo_ok(const Geo&, int stride) { return stride == 1; }

template <int CO, int CI>
WGeo whalo_geo(const Geo& g) {
  using T = WHalo<CO, CI>;
  WGeo w;
  w.n = g.n;
  w.d = g.d;
  w.h = g.h;
  w.w = g.w;
  w.od = g.od;
  w.oh = g.oh;
  w.ow = g.ow;
  w.ntx = (g.ow + 15) / 16;
  w.nty = (g.oh + T::TY - 1) / T::TY;
  w.ntz = (g.od + T::TZ - 1) / T::TZ;
  w.nbricks = w.ntx * w.nty * w.ntz * g.n;
  return w;
}

// the slice shape of a layer: 16 output channels, min(ci, 32) input channels
WGeo whalo_geo_of(const Geo& g) {
  return g.ci == 16 ? whalo_geo<16, 16>(g) : whalo_geo<16, 32>(g);
}

template <int CO, int CI>
void launch_whalo_c(const Geo& g, int up, const uint16_t* x, const uint16_t* dz, int nchunk, float* part,
                    float* dbpart, hipStream_t st) {
  const WGeo w = whalo_geo<CO, CI>(g);
  const dim3 grid(nchunk, (g.co / CO) * (g.ci / CI));
  constexpr bool PF = WHalo<CO, CI>::PF;
  if (up == 1)
    hipLaunchKernelGGL((k_conv_bwd_w_halo<CO, CI, 1, PF>), grid, dim3(192), 0, st, x, dz, w, g.co, g.ci, part,
                       dbpart);
  else
    hipLaunchKernelGGL((k_conv_bwd_w_halo<CO, CI, 2, PF>), grid, dim3(192), 0, st, x, dz, w, g.co, g.ci, part,
                       dbpart);
}

void launch_whalo(const Geo& g, int up, const uint16_t* x, const uint16_t* dz, int nchunk, float* part,
                  float* dbpart, hipStream_t st) {
  if (g.ci == 16) launch_whalo_c<16, 16>(g, up, x, dz, nchunk, part, dbpart, st);
  else launch_whalo_c<16, 32>(g, up, x, dz, nchunk, part, dbpart, st);
}

void wchunks(const Geo& g, int stride, int& nchunk, long long& vchunk) {
  if (whalo_ok(g, stride)) {  // one chunk per block of the brick walk, ~1024 blocks over the slices
    const long long nb = whalo_geo_of(g).nbricks;
    const int slices = (g.co / 16) * (g.ci / std::min(g.ci, 32));
    const int cap = kWHaloBlocks / slices;
    nchunk = (int)(nb < cap ? nb : cap);
    if (nchunk < 1) nchunk = 1;
    vchunk = 0;
    return;
  }
  const bool all_taps = (g.co / 16) * (g.ci / 16) <= kAllTapsMaxTiles;
  const long long target = all_taps ? 2048 : 76;
  long long vc = (g.mo + target - 1) / target;
  vc = ((vc + WV - 1) / WV) * WV;
  if (vc < WV) vc = WV;
  vchunk = vc;
  nchunk = (int)((g.mo + vc - 1) / vc);
  if (nchunk < 1) nchunk = 1;
}

int check_conv(int n, int d, int h, int w, int ci, int co, int stride, int up) {
  if (n < 1 || d < 1 || h < 1 || w < 1) return fail(SG_EINVAL, "empty extent");
  if (!chan_ok(ci) || !chan_ok(co)) return fail(SG_EINVAL, "channels must be 16, 32 or 64");
  if (!((stride == 1 || stride == 2) && (up == 1 || up == 2)) || (stride == 2 && up == 2))
    return fail(SG_EINVAL, "stride/upsample must be (1,1), (2,1) or (1,2)");
  return SG_OK;
}

}  // namespace

extern "C" {

const char* sg_last_error(void) { return g_err.c_str(); }

int sg_conv3d_fwd(const uint16_t* x, int n, int d, int h, int w, int ci, const uint16_t* wgt, const float* bias,
                  int co, int stride, int up, int relu, const uint16_t* skip, uint16_t* y, uint16_t* yr,
                  void* stream) {
  int rc = check_conv(n, d, h, w, ci, co, stride, up);
  if (rc) return rc;
  if (!x || !wgt || !bias || !y) return fail(SG_EINVAL, "null tensor");
  const Geo g = make_geo(n, d, h, w, ci, co, stride, up);
  hipStream_t st = (hipStream_t)stream;
  if (halo_fwd(ci, co, stride, up)) {
    if (up == 1)
      launch_halo<0>(n, d, h, w, co, x, wgt, bias, skip, nullptr, y, yr, relu, st);
    else if (co == 16)
      launch_halo_c<32, 16, 2, 0>(n, d, h, w, x, wgt, bias, skip, nullptr, y, yr, relu, st);
    else
      launch_halo_c<64, 32, 2, 0>(n, d, h, w, x, wgt, bias, skip, nullptr, y, yr, relu, st);
    return check_launch("sg_conv3d_fwd");
  }
  if (stride == 1 && up == 1) launch_fwd_su<1, 1>(g, x, wgt, bias, skip, y, yr, relu, st);
  else if (stride == 2) launch_fwd_su<2, 1>(g, x, wgt, bias, skip, y, yr, relu, st);
  else launch_fwd_su<1, 2>(g, x, wgt, bias, skip, y, yr, relu, st);
  return check_launch("sg_conv3d_fwd");
}

int sg_conv3d_bwd_data(const uint16_t* dz, int n, int d, int h, int w, int ci, const uint16_t* wgt_f, int co,
                       int stride, int up, const uint16_t* add, const uint16_t* mask, uint16_t* da, uint16_t* dzp,
                       void* stream) {
  int rc = check_conv(n, d, h, w, ci, co, stride, up);
  if (rc) return rc;
  if (!dz || !wgt_f || !dzp) return fail(SG_EINVAL, "null tensor");
  const Geo g = make_geo(n, d, h, w, ci, co, stride, up);
  hipStream_t st = (hipStream_t)stream;
  if (stride == 1 && up == 1 && ci == co && halo_data(ci)) {
    launch_halo<1>(n, d, h, w, ci, dz, wgt_f, nullptr, add, mask, dzp, da, 0, st);
    return check_launch("sg_conv3d_bwd_data");
  }
  if (stride == 2 && (g.mi >= (1LL << 31) || g.mo >= (1LL << 31)))
    return fail(SG_EINVAL, "stride-2 data gradient: more than 2^31 voxels");
  if (stride == 1 && up == 1) launch_bwd_data_su<1, 1>(g, dz, wgt_f, add, mask, da, dzp, st);
  else if (stride == 2 && g.ci == 16) launch_bwd_data_s2<16>(g, dz, wgt_f, add, mask, da, dzp, st);
  else if (stride == 2 && g.ci == 32) launch_bwd_data_s2<32>(g, dz, wgt_f, add, mask, da, dzp, st);
  else if (stride == 2) launch_bwd_data_s2<64>(g, dz, wgt_f, add, mask, da, dzp, st);
  else launch_bwd_data_su<1, 2>(g, dz, wgt_f, add, mask, da, dzp, st);
  return check_launch("sg_conv3d_bwd_data");
}

size_t sg_conv3d_bwd_weight_workspace(int n, int d, int h, int w, int ci, int co, int stride, int up) {
  if (check_conv(n, d, h, w, ci, co, stride, up)) return 0;
  const Geo g = make_geo(n, d, h, w, ci, co, stride, up);
  int nchunk;
  long long vchunk;
  wchunks(g, stride, nchunk, vchunk);
  return (size_t)nchunk * (27 * (size_t)co * ci + co) * sizeof(float);
}

int sg_conv3d_bwd_weight(const uint16_t* x, int n, int d, int h, int w, int ci, const uint16_t* dz, int co,
                         int stride, int up, void* ws, size_t ws_bytes, float* dw, float* db, void* stream) {
  int rc = check_conv(n, d, h, w, ci, co, stride, up);
  if (rc) return rc;
  if (!x || !dz || !ws || !dw || !db) return fail(SG_EINVAL, "null tensor");
  if (ws_bytes < sg_conv3d_bwd_weight_workspace(n, d, h, w, ci, co, stride, up))
    return fail(SG_EINVAL, "workspace too small");
  const Geo g = make_geo(n, d, h, w, ci, co, stride, up);
  int nchunk;
  long long vchunk;
  wchunks(g, stride, nchunk, vchunk);
  float* part = (float*)ws;
  float* dbpart = part + (size_t)nchunk * 27 * co * ci;
  hipStream_t st = (hipStream_t)stream;
  if (whalo_ok(g, stride)) launch_whalo(g, up, x, dz, nchunk, part, dbpart, st);
  else if (stride == 1 && up == 1) launch_bwd_w_su<1, 1>(g, x, dz, nchunk, vchunk, part, dbpart, st);
  else if (stride == 2) launch_bwd_w_su<2, 1>(g, x, dz, nchunk, vchunk, part, dbpart, st);
  else launch_bwd_w_su<1, 2>(g, x, dz, nchunk, vchunk, part, dbpart, st);
  const int nred = 27 * co * ci;
  hipLaunchKernelGGL(k_bwd_w_reduce, dim3((nred + 15) / 16 + (co + 15) / 16), dim3(256), 0, st, part, dbpart, nchunk,
                     co, ci, dw, db);
  return check_launch("sg_conv3d_bwd_weight");
}

int sg_fold_up_weights(const uint16_t* w, int co, int ci, uint16_t* wu, void* stream) {
  if (!w || !wu || !chan_ok(co) || !chan_ok(ci)) return fail(SG_EINVAL, "bad weights");
  const int n = ci * 64 * co;
  hipLaunchKernelGGL(k_fold_up_w, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, w, co, ci, wu);
  return check_launch("sg_fold_up_weights");
}

int sg_conv3d_bwd_data_up2(const uint16_t* dz, int n, int d, int h, int w, int ci, const uint16_t* wu, int co,
                           const uint16_t* add, const uint16_t* mask, uint16_t* da, uint16_t* dzp,
                           void* stream) {
  int rc = check_conv(n, d, h, w, ci, co, 1, 2);
  if (rc) return rc;
  if (!dz || !wu || !dzp) return fail(SG_EINVAL, "null tensor");
  const Geo g = make_geo(n, d, h, w, ci, co, 1, 2);
  hipStream_t st = (hipStream_t)stream;
  if (ci == 16) launch_bwd_data_up2<16>(g, dz, wu, add, mask, da, dzp, st);
  else if (ci == 32) launch_bwd_data_up2<32>(g, dz, wu, add, mask, da, dzp, st);
  else launch_bwd_data_up2<64>(g, dz, wu, add, mask, da, dzp, st);
  return check_launch("sg_conv3d_bwd_data_up2");
}

int sg_flip_weights(const uint16_t* w, int co, int ci, uint16_t* wf, void* stream) {
  if (!w || !wf || !chan_ok(co) || !chan_ok(ci)) return fail(SG_EINVAL, "bad weights");
  const int n = co * 27 * ci;
  hipLaunchKernelGGL(k_flip_w, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, w, co, ci, wf);
  return check_launch("sg_flip_weights");
}

int sg_adam(float* p, float* m, float* v, const float* g, long long count, int t, float lr, float beta1,
            float beta2, float eps, uint16_t* pb, void* stream) {
  if (!p || !m || !v || !g || count < 0 || t < 1) return fail(SG_EINVAL, "bad optimiser arguments");
  if (count == 0) return SG_OK;
  const float bc1 = (float)(1.0 - std::pow((double)beta1, t));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, t));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(count, 256)), dim3(256), 0, (hipStream_t)stream, p, m, v, g, count,
                     lr, beta1, beta2, eps, bc1, bc2, pb);
  return check_launch("sg_adam");
}

int sg_normalize(const float* x, int n, int c, long long vox, const float* shift, const float* scale, float* xn,
                 void* stream) {
  if (!x || !shift || !scale || !xn || n < 1 || c < 1 || vox < 1) return fail(SG_EINVAL, "bad normalize");
  const long long total = (long long)n * c * vox;
  hipLaunchKernelGGL(k_normalize, dim3(blocks_for(total, 256)), dim3(256), 0, (hipStream_t)stream, x, c, vox,
                     total, shift, scale, xn);
  return check_launch("sg_normalize");
}

int sg_pack(const float* xn, int n, int c, long long vox, int cpad, uint16_t* xb, void* stream) {
  if (!xn || !xb || n < 1 || c < 1 || vox < 1 || !chan_ok(cpad) || cpad < c) return fail(SG_EINVAL, "bad pack");
  const long long nvox = (long long)n * vox;
  hipLaunchKernelGGL(k_pack, dim3(blocks_for(nvox, 256)), dim3(256), 0, (hipStream_t)stream, xn, c, vox, cpad,
                     nvox, xb);
  return check_launch("sg_pack");
}

int sg_residual_loss(const float* xn, const float* tn, const uint16_t* r, const float* rs, int n, int c,
                     long long vox, int cpad, float mass_weight, uint16_t* dr, double* loss, void* ws,
                     void* stream) {
  if (!xn || !tn || !r || !dr || !ws || n < 1 || c < 1 || vox < 1 || !chan_ok(cpad) || cpad < c ||
      !(mass_weight >= 0.0f))
    return fail(SG_EINVAL, "bad loss arguments");
  if (mass_weight > 0.0f && n > kLossMaxSamples) return fail(SG_EINVAL, "mass term: too many samples");
  const long long nvox = (long long)n * vox;
  const double count = (double)n * c * vox;
  hipStream_t st = (hipStream_t)stream;
  double* part = (double*)ws;
  double* msum = mass_weight > 0.0f ? part + kLossBlocks : nullptr;
  if (msum) {  // the mass partials use the loss-partials region before the loss kernel fills it
    const int np = std::min(64, std::max(1, kLossBlocks / n));
    hipLaunchKernelGGL(k_mass_residual, dim3(np, n), dim3(256), 0, st, xn, tn, r, rs, c, vox, cpad, np, part);
    hipLaunchKernelGGL(k_mass_final, dim3((n + 63) / 64), dim3(64), 0, st, part, n, np, msum);
  }
  // d/dd of mw * mean_n (S_n / V)^2 is 2 mw S_n / (n V^2)
  const float mgrad = (float)(2.0 * mass_weight / ((double)n * (double)vox * (double)vox));
  hipLaunchKernelGGL(k_residual_loss, dim3(kLossBlocks), dim3(256), 0, st, xn, tn, r, rs, c, vox, cpad, nvox,
                     (float)(1.0 / count), msum, mgrad, dr, part);
  if (loss)
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, part, kLossBlocks, 1.0 / count, msum, n,
                       (double)vox, (double)mass_weight, loss);
  return check_launch("sg_residual_loss");
}

int sg_unpack(const float* xn, const uint16_t* r, const float* rs, int n, int c, long long vox, int cpad,
              const float* shift, const float* scale, float* out, void* stream) {
  if (!xn || !r || !shift || !scale || !out || n < 1 || c < 1 || vox < 1 || !chan_ok(cpad) || cpad < c)
    return fail(SG_EINVAL, "bad unpack");
  const long long total = (long long)n * c * vox;
  hipLaunchKernelGGL(k_unpack, dim3(blocks_for(total, 256)), dim3(256), 0, (hipStream_t)stream, xn, r, rs, c, vox,
                     cpad, total, shift, scale, out);
  return check_launch("sg_unpack");
}

int sg_coarsen(const float* phi, const float* u, const float* p, int nx, int ny, int nz, int z0c, int dw,
               float* out, void* stream) {
  if (!phi || !u || !p || !out || nx < 2 || ny < 2 || nz < 2 || (nx & 1) || (ny & 1) || z0c < 0 || dw < 1)
    return fail(SG_EINVAL, "bad coarsen");
  const long long total = 5LL * dw * (nx / 2) * (ny / 2);
  hipLaunchKernelGGL(k_coarsen, dim3(blocks_for(total, 256)), dim3(256), 0, (hipStream_t)stream, phi, u, p, nx, ny,
                     nz, z0c, dw, out);
  return check_launch("sg_coarsen");
}

int sg_phi_budget(const float* x, int n, int c, int d, int h, int w, double* sums, void* stream) {
  if (!x || !sums || n < 1 || c < 4 || d < 1 || h < 1 || w < 1) return fail(SG_EINVAL, "bad budget");
  hipLaunchKernelGGL(k_phi_budget, dim3(n), dim3(256), 0, (hipStream_t)stream, x, c, d, h, w, sums);
  return check_launch("sg_phi_budget");
}

int sg_gather(const float* store, long long rows, long long len, const long long* idx, int n, float* out,
              void* stream) {
  if (!store || !idx || !out || rows < 1 || len < 1 || n < 0) return fail(SG_EINVAL, "bad gather");
  if (n == 0) return SG_OK;
  hipLaunchKernelGGL(k_gather, dim3(blocks_for((long long)n * len, 256)), dim3(256), 0, (hipStream_t)stream,
                     store, rows, len, idx, n, out);
  return check_launch("sg_gather");
}

}  // extern "C"
