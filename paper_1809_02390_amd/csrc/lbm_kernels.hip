// HIP kernels and C-ABI entry points of the self-tuning-EOS D2Q9 library
// (gfx950).  See include/lbm.h for the contract of every entry point.
//
// Data layout, x fastest.  State buffers (state_layout) interleave rows,
// population i of node (x, y) at element (9 y + i) nx + x (FP32 states
// larger than 4 GiB are read with band-relative or 64-bit offsets,
// wide_state).  The adjoint state interleaves its eleven fields the same
// way when its offsets fit 32 bits, else it holds eleven planes P =
// plane_elems apart (nx*ny rounded up to 64 plus a pad, so that the planes
// do not start at one offset modulo a large power of two); the 2-byte
// reference densities and the caller's plain arrays hold planes of nx*ny.  Two caller-owned
// buffers A and B alternate; the buffer that is
// read by the next step holds the post-collision populations of the previous
// step at their source node ("pull" streaming: f_i(x, t) = src_i(x - e_i)).
//
// Storages (one template parameter of every kernel):
//   F32   f-bar stored as float;
//   F16 / BF16  f-bar stored in two bytes as S (f-bar - f_ref), with f_ref the
//         rest equilibrium at the reference density rho~ of the node the
//         population streams to.  rho~ is that node's density of the previous
//         step in binary16, kept in two planes that alternate like A and B.
//         The encoder takes the neighbour densities from the LDS tile it
//         already holds for the force stencil; the decoder reads its own rho~.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>

#include "lbm.h"
#include "lbm_cell.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_OK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Velocity set (supplement Eq. 3) as compile-time tables
// ---------------------------------------------------------------------------
constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// ---------------------------------------------------------------------------
// Storage policies
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_f16(float v) { return __half_as_ushort(__float2half_rn(v)); }
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return __half2float(__ushort_as_half(h)); }

// binary32 -> bfloat16, round to nearest even (one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t f32_to_bf16(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// The reference density rho~ of a node: its density rounded to binary16.
__device__ __forceinline__ float ref_density(float rho) { return f16_to_f32(f32_to_f16(rho)); }

struct StoreF32 {
  using E = float;
  static constexpr int ES = 4;
  static constexpr bool kRef = false;
};

template <int KIND>
struct Store16 {
  using E = uint16_t;
  static constexpr int ES = 2;
  static constexpr bool kRef = true;
  __device__ static float to_f32(uint16_t h) { return KIND == LBM_FP16 ? f16_to_f32(h) : bf16_to_f32(h); }
  __device__ static uint16_t from_f32(float v) { return KIND == LBM_FP16 ? f32_to_f16(v) : f32_to_bf16(v); }
};

// ---------------------------------------------------------------------------
// Addressing: per-plane base pointers (uniform) and 32-bit byte offsets
// ---------------------------------------------------------------------------
// i mod n.  Tile coordinates lie within one period of [0, n) except on
// lattices narrower than a tile, which alone take the integer division.
__device__ __forceinline__ int wrap(int i, int n) {
  if (i >= n)
    i -= n;
  else if (i < 0)
    i += n;
  if ((unsigned)i >= (unsigned)n) {
    i %= n;
    if (i < 0) i += n;
  }
  return i;
}

// Row offsets (row * rp * ES, rp the row pitch) of rows y, y-1, y+1 and column offsets
// (x * ES) of columns x, x-1, x+1 of a node, periodic.
template <int ES>
struct NodeAddr {
  unsigned r0, rm, rp, c0, cm, cp;
};

// One multiplication per node; the neighbours' offsets are the node's plus
// or minus one row (column), or the opposite edge.
template <int ES>
__device__ __forceinline__ NodeAddr<ES> node_addr(int x, int y, int nx, int ny, unsigned rp, int yb = 0) {
  // rows relative to row yb; with yb > 0 (band addressing) y never wraps
  const unsigned rb = ES * rp, r0 = rb * (unsigned)(y - yb), rlast = rb * (unsigned)(ny - 1 - yb);
  const unsigned c0 = ES * (unsigned)x, clast = ES * (unsigned)(nx - 1);
  return {r0, y == 0 ? rlast : r0 - rb, y == ny - 1 ? rb * (unsigned)(-yb) : r0 + rb,
          c0, x == 0 ? clast : c0 - ES, x == nx - 1 ? 0u : c0 + ES};
}

template <typename E>
__device__ __forceinline__ E ldb(const char* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const E*>(base + off);
}

template <typename E>
struct Planes {
  const char* p[9];
};

template <typename E>
__device__ __forceinline__ Planes<E> planes(const void* src, size_t N) {
  Planes<E> P;
#pragma unroll
  for (int i = 0; i < 9; ++i) P.p[i] = reinterpret_cast<const char*>(reinterpret_cast<const E*>(src) + (size_t)i * N);
  return P;
}

template <typename E>
struct OutPlanes {
  char* p[9];
};

template <typename E>
__device__ __forceinline__ OutPlanes<E> out_planes(void* dst, size_t N) {
  OutPlanes<E> P;
#pragma unroll
  for (int i = 0; i < 9; ++i) P.p[i] = reinterpret_cast<char*>(reinterpret_cast<E*>(dst) + (size_t)i * N);
  return P;
}

// Elements from one plane of an internal buffer (A/B state, checkpoint,
// adjoint state) to the next: nx*ny rounded up to 64, plus LBM_PLANE_PAD
// bytes, so that the planes do not all start at one offset modulo a large
// power of two (the streams of the nine planes then spread over the HBM
// channels).  The 2-byte reference planes and the caller's plain arrays use
// nx*ny.
#ifndef LBM_PLANE_PAD
#define LBM_PLANE_PAD 16640
#endif
__host__ __device__ __forceinline__ size_t plane_elems(int nx, int ny, int es) {
  return ((size_t)nx * ny + 63) / 64 * 64 + (size_t)(LBM_PLANE_PAD / es);
}

// Layout of a state buffer (A/B, checkpoint): elements from one population
// to the next (ps) and from one lattice row to the next (rp).  States
// interleave rows -- the nine populations of a lattice row are nine
// consecutive buffer rows, population i of node (x, y) at (9 y + i) nx + x.
// A wave's nine loads (stores) of a row segment then fall within 9 nx
// elements instead of nine planes apart, which keeps more of them in open
// DRAM pages (a data-movement kernel with the step's access pattern moves
// 3-6 % more bytes per second; the FP32 step gains 7 % at 4096^2, the
// 2-byte steps 1 %).
struct Layout {
  size_t ps;    // elements between populations
  unsigned rp;  // elements between lattice rows
};
__host__ __device__ __forceinline__ Layout state_layout(int nx, int, int) { return {(size_t)nx, 9u * (unsigned)nx}; }

// Byte offsets of a state from uniform bases fit the 32-bit lane offsets
// when 9 es nx ny < 2^32 (always for the 2-byte storages; FP32 lattices up
// to 119M nodes): kAbs.  Larger FP32 states are read per tile relative to
// the band of rows the tile reads (kBand: tile rows whose halo stays inside
// the lattice) or with 64-bit addresses (kWide: the tile rows that wrap),
// in two launches, so that the wide path adds no registers to the kernel
// that runs nearly every tile.
enum { kAbs = 0, kBand = 1, kWide = 2 };
__host__ __device__ __forceinline__ bool wide_state(int nx, int ny, int es) {
  return 9ull * (unsigned long long)es * (unsigned long long)nx * (unsigned long long)ny > 0xFFFFFFFFull;
}

// Tile rows of one launch: local tile row r is row r0 + r for r < na, else
// r1 + (r - na) (the wide launch takes the rows at both ends).
struct TileRows {
  int r0, na, r1;
};
__device__ __forceinline__ int tile_row(const TileRows& t, int r) { return r < t.na ? t.r0 + r : t.r1 + (r - t.na); }

// Layout of an adjoint state buffer: eleven fields (L_0..L_8, A_x, A_y)
// with rows interleaved like the FP32 state when every byte offset fits 32
// bits (44 nx ny < 2^32), else eleven planes plane_elems apart.
__host__ __device__ __forceinline__ Layout adj_layout(int nx, int ny) {
  if (44ull * (unsigned long long)nx * (unsigned long long)ny <= 0xFFFFFFFFull)
    return {(size_t)nx, 11u * (unsigned)nx};
  return {plane_elems(nx, ny, 4), (unsigned)nx};
}

// Raw stored values arriving at a node: raw_i = src_i(x - e_i).
template <typename E>
__device__ __forceinline__ void pull_raw(const Planes<E>& P, const NodeAddr<sizeof(E)>& a, E* r) {
  r[0] = ldb<E>(P.p[0], a.r0 + a.c0);
  r[1] = ldb<E>(P.p[1], a.r0 + a.cm);
  r[2] = ldb<E>(P.p[2], a.rm + a.c0);
  r[3] = ldb<E>(P.p[3], a.r0 + a.cp);
  r[4] = ldb<E>(P.p[4], a.rp + a.c0);
  r[5] = ldb<E>(P.p[5], a.rm + a.cm);
  r[6] = ldb<E>(P.p[6], a.rm + a.cp);
  r[7] = ldb<E>(P.p[7], a.rp + a.cp);
  r[8] = ldb<E>(P.p[8], a.rp + a.cm);
}

// Populations arriving at node (x, y) from a row-interleaved FP32 state,
// any node (periodic wrap), with 64-bit addresses (kWide).
__device__ __forceinline__ void pull_rows(const char* __restrict__ base, int x, int y, int nx, int ny, float* r) {
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int row[9] = {y, y, ym, y, yp, ym, ym, yp, yp};  // source of population i: (x, y) - e_i
  const int col[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
#pragma unroll
  for (int i = 0; i < 9; ++i)
    r[i] = *reinterpret_cast<const float*>(base + 4 * (((size_t)row[i] * 9 + i) * nx + col[i]));
}

// Decode the raw values of a node into f_i (FP32).  rref is the node's
// stored reference density (binary16 bits; ignored for F32).
template <class St>
__device__ __forceinline__ void decode(const typename St::E* r, uint16_t rref, const RefPoly<float>& q, float* f) {
  if constexpr (St::kRef) {
    const float rt = f16_to_f32(rref);
    const float ref[3] = {ref_value(q, 0, rt), ref_value(q, 1, rt), ref_value(q, 2, rt)};
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = ref[velocity_class(i)] + St::to_f32(r[i]) * q.inv_scale;
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = r[i];
  }
}

// Encode f-bar_i of one node given the reference densities of the nine
// nodes its populations stream to (index i: x + e_i).
template <class St>
__device__ __forceinline__ void encode(const float* f, const float* rdest, const RefPoly<float>& q,
                                       typename St::E* out) {
  if constexpr (St::kRef) {
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = St::from_f32((f[i] - ref_value(q, velocity_class(i), rdest[i])) * q.scale);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = f[i];
  }
}

// ---------------------------------------------------------------------------
// Tiles: TX x TY nodes per workgroup of TX x WY threads; each thread owns
// NPT = TY/WY nodes of one column.  The tile plus a one-node ring of
// densities is staged in LDS for the force stencil; ring nodes pull their
// own populations (L2 hits: neighbouring tiles run on the same XCD).
// ---------------------------------------------------------------------------
template <int TX_, int TY_, int WY_>
struct TileShape {
  static constexpr int TX = TX_, TY = TY_, WY = WY_, NPT = TY / WY, LW = TX + 2;
  static constexpr int NRING = 2 * LW + 2 * TY, NTHREADS = TX * WY, LDS = (TY + 2) * LW;
  static_assert(TY % WY == 0, "rows per thread");
  static_assert(NRING <= NTHREADS, "one ring node per thread");
};

// Tiles of the step kernel (TX, TY, WY), per storage; compile-time tuning
// knobs.  FP32 (bound by HBM): 256 x 8 in 1024-thread workgroups, 2-byte
// storages (bound by the vector ALU): 128 x 8 in 512.
#ifndef LBM_STEP_TILE_F32
#define LBM_STEP_TILE_F32 256, 8, 4
#endif
#ifndef LBM_STEP_TILE_16
#define LBM_STEP_TILE_16 128, 8, 4
#endif
template <class St>
struct StepTileOf {
  using type = TileShape<LBM_STEP_TILE_16>;
};
template <>
struct StepTileOf<StoreF32> {
  using type = TileShape<LBM_STEP_TILE_F32>;
};
template <class St>
using StepTile = typename StepTileOf<St>::type;
using MomTile = TileShape<64, 16, 4>;

// Tile order across the eight XCDs of the chip: workgroups are dealt to the
// XCDs round-robin by dispatch index, so dispatch b runs on XCD b % 8.  Give
// each XCD one contiguous run of tiles (in raster order) so that the tiles
// whose halo lines overlap share that XCD's L2.  A bijection onto
// [0, ntiles) for any ntiles.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int q = ntiles >> 3, r = ntiles & 7, xcd = b & 7, local = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + local;
}

// Position (tx, ty) of the tile with order index t when the tiles are
// visited in vertical strips of `strip` tile columns (1 <= strip <= ntx),
// band by band within a strip: the tile that shares a halo line with the
// tile above it comes `strip` tiles later, whatever the lattice width, so
// the line is still in L2 when it is read again.  A bijection for any ntx,
// nty.
__device__ __forceinline__ void strip_tile(int t, int ntx, int nty, int strip, int& tx, int& ty) {
  const int full = ntx / strip, per = strip * nty;  // full strips first, then a narrower one
  if (t < full * per) {
    const int s = t / per, rem = t - s * per;
    ty = rem / strip;
    tx = s * strip + (rem - ty * strip);
  } else {
    const int w = ntx - full * strip, rem = t - full * per;
    ty = rem / w;
    tx = full * strip + (rem - ty * w);
  }
}

// Coordinates (hx, hy) in the (TY+2) x LW density tile of ring slot t:
// slots [0, LW) the top row, [LW, 2 LW) the bottom row, then the left and
// the right column (TY nodes each).  Selects rather than branches: every
// ring thread of a wave takes the same instructions.
template <class S>
__device__ __forceinline__ void ring_slot(int t, int& hx, int& hy) {
  const bool row = t < 2 * S::LW, bottom = t >= S::LW, right = t >= 2 * S::LW + S::TY;
  const int c = t - 2 * S::LW - (right ? S::TY : 0);  // column slots: row index - 1
  hx = row ? (bottom ? t - S::LW : t) : (right ? S::LW - 1 : 0);
  hy = row ? (bottom ? S::TY + 1 : 0) : c + 1;
}

// Stored values of one tile held in registers: NPT own nodes per thread and,
// for the first NRING threads, one ring node; plus their reference densities.
template <class S, class St>
struct TileRegs {
  typename St::E raw[S::NPT][9];
  typename St::E rraw[9];
  uint16_t rref[S::NPT];
  uint16_t rrref;
};

// Whether the tile at (x0, y0), its ring and the ring's pull sources lie
// inside the lattice without wrapping (the common case on large lattices).
template <class S>
__device__ __forceinline__ bool interior_tile(int x0, int y0, int nx, int ny) {
  return x0 >= 2 && y0 >= 2 && x0 + S::TX + 2 <= nx && y0 + S::TY + 2 <= ny;
}

// Issue the loads of the tile at (x0, y0); ring loads first.  P holds the
// population bases of lattice row yb (0, or the tile's band origin y0 - 2
// for kBand); offsets count rows from there.  kInterior (interior_tile
// true): every population's pull shift goes into its uniform base, so the
// nine loads of a node share one offset register.  kWideAddr: 64-bit
// addresses from the state's base P.p[0] (FP32, rows that wrap).
template <class S, class St, bool kInterior = false, bool kWideAddr = false>
__device__ __forceinline__ void issue_tile(const Planes<typename St::E>& P, const uint16_t* __restrict__ rho_ref,
                                           int nx, int ny, int x0, int y0, int yb, TileRegs<S, St>& R) {
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * S::TX + tx;
  if constexpr (kWideAddr) {
    static_assert(sizeof(typename St::E) == 4 && !St::kRef, "64-bit addressing is for FP32 states");
    if (tid < S::NRING) {
      int hx, hy;
      ring_slot<S>(tid, hx, hy);
      pull_rows(P.p[0], wrap(x0 + hx - 1, nx), wrap(y0 + hy - 1, ny), nx, ny, R.rraw);
    }
    const int xw = wrap(x0 + tx, nx);
#pragma unroll
    for (int k = 0; k < S::NPT; ++k) pull_rows(P.p[0], xw, wrap(y0 + ty + k * S::WY, ny), nx, ny, R.raw[k]);
    return;
  } else if constexpr (kInterior) {
    using E = typename St::E;
    const unsigned rb = St::ES * state_layout(nx, ny, St::ES).rp;
    Planes<E> Q;  // Q_i + offset(x) = P_i + offset(x - e_i)
#pragma unroll
    for (int i = 0; i < 9; ++i) Q.p[i] = P.p[i] - (ptrdiff_t)kCy[i] * rb - kCx[i] * St::ES;
    const char* rref = reinterpret_cast<const char*>(rho_ref);  // reference plane, row pitch 2 nx bytes
    if (tid < S::NRING) {
      int hx, hy;
      ring_slot<S>(tid, hx, hy);
      const unsigned off = (unsigned)(y0 + hy - 1 - yb) * rb + (unsigned)(x0 + hx - 1) * St::ES;
#pragma unroll
      for (int i = 0; i < 9; ++i) R.rraw[i] = ldb<E>(Q.p[i], off);
      if constexpr (St::kRef) R.rrref = ldb<uint16_t>(rref, 2u * ((unsigned)(y0 + hy - 1) * nx + (unsigned)(x0 + hx - 1)));
    }
    const unsigned off0 = (unsigned)(y0 + ty - yb) * rb + (unsigned)(x0 + tx) * St::ES;
#pragma unroll
    for (int k = 0; k < S::NPT; ++k) {
      const unsigned off = off0 + (unsigned)(k * S::WY) * rb;
#pragma unroll
      for (int i = 0; i < 9; ++i) R.raw[k][i] = ldb<E>(Q.p[i], off);
      if constexpr (St::kRef) R.rref[k] = ldb<uint16_t>(rref, 2u * ((unsigned)(y0 + ty + k * S::WY) * nx + (unsigned)(x0 + tx)));
    }
    // Distinct markers end the two load paths, so the compiler cannot sink
    // their last loads into the join (which would force 64-bit per-lane
    // addresses on this path).
    asm volatile("; tile loads issued: interior" ::: "memory");
    return;
  }
  if (tid < S::NRING) {
    int hx, hy;
    ring_slot<S>(tid, hx, hy);
    const int gx = wrap(x0 + hx - 1, nx), gy = wrap(y0 + hy - 1, ny);
    pull_raw<typename St::E>(P, node_addr<St::ES>(gx, gy, nx, ny, state_layout(nx, ny, St::ES).rp, yb), R.rraw);
    if constexpr (St::kRef) R.rrref = ldb<uint16_t>(reinterpret_cast<const char*>(rho_ref), 2u * ((unsigned)gy * nx + (unsigned)gx));
  }
  const int xw = wrap(x0 + tx, nx);
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    const int yw = wrap(y0 + ty + k * S::WY, ny);
    pull_raw<typename St::E>(P, node_addr<St::ES>(xw, yw, nx, ny, state_layout(nx, ny, St::ES).rp, yb), R.raw[k]);
    if constexpr (St::kRef) R.rref[k] = ldb<uint16_t>(reinterpret_cast<const char*>(rho_ref), 2u * ((unsigned)yw * nx + (unsigned)xw));
  }
  asm volatile("; tile loads issued: edge" ::: "memory");
}

// The three class values of the reference equilibrium at the reference
// density of a tile node (2-byte storages), times -S, staged for the
// encoders of the node's neighbours: sref[class * LDS + pos] (the encoder
// is then one fused multiply-add, S f + (-S f_ref)).
template <class S>
__device__ __forceinline__ void stage_ref(const RefPoly<float>& q, float rho, int pos, float* sref) {
  const float rt = ref_density(rho);
#pragma unroll
  for (int c = 0; c < 3; ++c) sref[c * S::LDS + pos] = -q.scale * ref_value(q, c, rt);
}

// Decode the tile, stage densities of the tile and its ring into
// srho[(TY+2)][LW], keep the own nodes' populations and densities in
// registers.
template <class S, class St>
__device__ __forceinline__ void stage_tile(const TileRegs<S, St>& R, const RefPoly<float>& q,
                                           float (&f)[S::NPT][9], float (&rho)[S::NPT], float* srho,
                                           float* sref) {
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * S::TX + tx;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    decode<St>(R.raw[k], St::kRef ? R.rref[k] : 0, q, f[k]);
    rho[k] = density(f[k]);
    const int pos = (ty + k * S::WY + 1) * S::LW + tx + 1;
    srho[pos] = rho[k];
    if (St::kRef && sref) stage_ref<S>(q, rho[k], pos, sref);
  }
  if (tid < S::NRING) {
    int hx, hy;
    ring_slot<S>(tid, hx, hy);
    float fr[9];
    decode<St>(R.rraw, St::kRef ? R.rrref : 0, q, fr);
    const float r = density(fr);
    srho[hy * S::LW + hx] = r;
    if (St::kRef && sref) stage_ref<S>(q, r, hy * S::LW + hx, sref);
  }
}

// The stencil neighbours of tile position (hx, hy), indexed like the
// populations: nb[i] = rho(x + e_i) (nb[0] = rho(x)).
template <class S>
__device__ __forceinline__ void neighbours(const float* srho, int hx, int hy, float* nb) {
  const float* r = srho + hy * S::LW + hx;
#pragma unroll
  for (int i = 0; i < 9; ++i) nb[i] = r[kCy[i] * S::LW + kCx[i]];
}

// Step kernel: one tile per workgroup, tiles ordered across the XCDs by
// xcd_tile so that neighbouring tiles (whose halo lines overlap) run on the
// same XCD and share its L2.
template <class S, class St, int kMode = kAbs>
__global__ __launch_bounds__(S::NTHREADS) void step_kernel(const void* __restrict__ src, void* __restrict__ dst,
                                                           const uint16_t* __restrict__ ref_in,
                                                           uint16_t* __restrict__ ref_out, int nx, int ny, int ntx,
                                                           int ntiles, int strip, Coef<float> c, RefPoly<float> q,
                                                           TileRows rows) {
  using E = typename St::E;
  __shared__ float srho[S::LDS];
  __shared__ float sref[St::kRef ? 3 * S::LDS : 1];
  const Layout L = state_layout(nx, ny, St::ES);
  const size_t N = L.ps, rowb = (size_t)St::ES * L.rp;
  int tx, ty;
  strip_tile(xcd_tile(blockIdx.x, ntiles), ntx, ntiles / ntx, strip, tx, ty);
  const int x0 = tx * S::TX, y0 = tile_row(rows, ty) * S::TY;
  float f[S::NPT][9];
  float rho[S::NPT];
  {
    TileRegs<S, St> R;
    const int yb = kMode == kBand ? y0 - 2 : 0;  // loads: rows counted from yb
    const char* sb = static_cast<const char*>(src) + (size_t)yb * rowb;
    if constexpr (kMode == kWide)
      issue_tile<S, St, false, true>(planes<E>(src, N), ref_in, nx, ny, x0, y0, 0, R);
    else if (interior_tile<S>(x0, y0, nx, ny))
      issue_tile<S, St, true>(planes<E>(sb, N), ref_in, nx, ny, x0, y0, yb, R);
    else
      issue_tile<S, St, false>(planes<E>(sb, N), ref_in, nx, ny, x0, y0, yb, R);
    stage_tile<S, St>(R, q, f, rho, srho, St::kRef ? sref : nullptr);
  }
  __syncthreads();
  const int x = x0 + threadIdx.x;
  if (x >= nx) return;
  // stores: rows counted from row 0 (kAbs) or from the tile's first row
  const int ys = kMode == kAbs ? 0 : y0;
  const OutPlanes<E> Q = out_planes<E>(static_cast<char*>(dst) + (size_t)ys * rowb, N);
  const unsigned rb = St::ES * L.rp;
  const unsigned o0 = rb * (unsigned)(y0 - ys + threadIdx.y) + St::ES * (unsigned)x;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    const int ly = threadIdx.y + k * S::WY, y = y0 + ly;
    if (y >= ny) break;
    float nb[9];
    neighbours<S>(srho, threadIdx.x + 1, ly + 1, nb);
    float gx, gy;
    stencil(nb[1], nb[2], nb[3], nb[4], nb[5], nb[6], nb[7], nb[8], gx, gy);
    collide_node<float, St::kRef>(f[k], rho[k], gx, gy, c);
    E out[9];
    if constexpr (St::kRef) {
      // f-bar_i streams to x + e_i: encode it against that node's reference
      const int pos = (ly + 1) * S::LW + threadIdx.x + 1;
#pragma unroll
      for (int i = 0; i < 9; ++i)
        out[i] = St::from_f32(fmaf(f[k][i], q.scale, sref[velocity_class(i) * S::LDS + pos + kCy[i] * S::LW + kCx[i]]));
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) out[i] = f[k][i];
    }
    const unsigned o = o0 + (unsigned)(k * S::WY) * rb;
    if constexpr (St::kRef)  // 2 nx ny < 2^32 for every 2-byte state: a 32-bit offset from the plane
      *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(ref_out) + 2u * ((unsigned)y * nx + (unsigned)x)) =
          f32_to_f16(nb[0]);
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(out[i], reinterpret_cast<E*>(Q.p[i] + o));
  }
}

// ---------------------------------------------------------------------------
// Two time steps per launch (FP32 storage).  A workgroup advances a TX x TY
// tile from the state of time t to that of t + 2 without storing t + 1:
//   (A) pull f(t) onto the tile plus a three-node ring and stage the
//       densities of that region in LDS;
//   (B) collide the tile plus a two-node ring (step t), streaming each
//       post-collision population in LDS to the node it arrives at, if that
//       node lies on the tile or its one-node ring;
//   (C) form the densities of the tile and its ring at t + 1;
//   (D) collide the tile (step t + 1) and store f-bar.
// Every node is updated by the operations of step_kernel in the same order
// (density, stencil, collide_node), so two fused steps give the bits of two
// single steps.  Per two lattice updates the tile moves 36 B of each node in
// and 36 B out, half the bytes of two single steps, for (TX+4)(TY+4)
// collisions instead of TX TY in step t (64 x 24 tiles: 12 % more per
// update over the two steps), so the kernel is bound by the vector ALU
// rather than by HBM.  The tile is 64 x 24 in 512 threads (70 KB of LDS, two
// workgroups per CU; measured at 4096^2 against 64 x 16 in 256 or 512
// threads, 32 x 32, 64 x 20, 64 x 32, 128 x 16 and other thread counts).
// kMid also stores the state of t + 1 (the checkpoint driver keeps every
// state).
// ---------------------------------------------------------------------------
template <int TX_, int TY_, int WY_>
struct Tile2Shape {
  static constexpr int TX = TX_, TY = TY_, WY = WY_, NTHREADS = TX * WY;
  static constexpr int W1 = TX + 6, H1 = TY + 6;  // loaded region: the tile and a three-node ring
  static constexpr int KA = (H1 + WY - 1) / WY;   // loaded nodes of the tile's columns per thread
  static constexpr int NSIDE = 6 * H1;            // loaded nodes left and right of the tile's columns
  static constexpr int KD = TY / WY;              // tile nodes per thread
  // the tile and its one-node ring (positions as in TileShape: LW, ring_slot)
  static constexpr int LW = TX + 2, NRING = 2 * LW + 2 * TY, G = (TY + 2) * LW;
  static_assert(TY % WY == 0, "rows per thread");
  static_assert(NSIDE <= NTHREADS && NRING <= NTHREADS, "one side node and one ring node per thread");
};
#ifndef LBM_STEP2_TILE
#define LBM_STEP2_TILE 64, 24, 8
#endif
using Step2Tile = Tile2Shape<LBM_STEP2_TILE>;

// Whether the loaded region of the tile at (x0, y0) and its pull sources lie
// inside the lattice without wrapping.
template <class S>
__device__ __forceinline__ bool interior_tile2(int x0, int y0, int nx, int ny) {
  return x0 >= 4 && y0 >= 4 && x0 + S::TX + 4 <= nx && y0 + S::TY + 4 <= ny;
}

// Stencil gradient at position pos of an LDS density tile lw nodes wide.
template <int LWD>
__device__ __forceinline__ void stencil_at(const float* s, int pos, float& gx, float& gy) {
  float nb[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) nb[i] = s[pos + kCy[i] * LWD + kCx[i]];
  stencil(nb[1], nb[2], nb[3], nb[4], nb[5], nb[6], nb[7], nb[8], gx, gy);
}

// Stream the post-collision populations of the node at position (X, Y) of
// the loaded region to the tile-plus-ring positions they arrive at: sg[i G +
// (Y - 2 + e_iy) LW + X - 2 + e_ix], skipped where that lies outside.
template <class S, bool kCheckX>
__device__ __forceinline__ void push_node(const float* f, int X, int Y, float* sg) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int X2 = X - 2 + kCx[i], Y2 = Y - 2 + kCy[i];
    const bool in = (unsigned)Y2 < (unsigned)(S::TY + 2) && (!kCheckX || (unsigned)X2 < (unsigned)S::LW);
    if (in) sg[i * S::G + Y2 * S::LW + X2] = f[i];
  }
}

template <class S, bool kMid>
__global__ __launch_bounds__(S::NTHREADS) void step2_kernel(const float* __restrict__ src, float* __restrict__ mid,
                                                            float* __restrict__ dst, int nx, int ny, int ntx,
                                                            int ntiles, int strip, Coef<float> c) {
  __shared__ float s1[S::W1 * S::H1];  // densities at t of the loaded region; then at t + 1 of tile + ring
  __shared__ float sg[9 * S::G];       // populations arriving at the tile and its ring at t + 1
  const size_t rowb = (size_t)36 * nx;  // bytes from one lattice row of a state to the next
  // rb: the same in 32 bits (offsets within a tile's rows); pb: bytes from
  // one population of a row to the next
  const unsigned rb = 36u * (unsigned)nx, pb = 4u * (unsigned)nx;
  int tx, ty;
  strip_tile(xcd_tile(blockIdx.x, ntiles), ntx, ntiles / ntx, strip, tx, ty);
  const int x0 = tx * S::TX, y0 = ty * S::TY;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * S::TX + lx;
  // side node of this thread: column sc of the six outside the tile's columns
  const int sY = tid / 6, sc = tid - 6 * sY, sX = sc < 3 ? sc : S::TX + sc;
  const bool side = tid < S::NSIDE;
  float fa[S::KA][9], fs[9];
  // (A) f(t) arriving at the loaded region, position (X, Y) = node (x0 - 3 + X, y0 - 3 + Y)
  if (interior_tile2<S>(x0, y0, nx, ny)) {
    // rows counted from y0 - 4; each population's pull shift in its uniform base
    const char* sb = reinterpret_cast<const char*>(src) + (size_t)(y0 - 4) * rowb;
    const char* Q[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = sb + (ptrdiff_t)i * pb - (ptrdiff_t)kCy[i] * rb - kCx[i] * 4;
    const unsigned o0 = (unsigned)(ly + 1) * rb + 4u * (unsigned)(x0 + lx);
#pragma unroll
    for (int k = 0; k < S::KA; ++k)
      if (k * S::WY < S::H1 - (S::WY - 1) || ly + k * S::WY < S::H1) {
        const unsigned o = o0 + (unsigned)(k * S::WY) * rb;
#pragma unroll
        for (int i = 0; i < 9; ++i) fa[k][i] = ldb<float>(Q[i], o);
      }
    if (side) {
      const unsigned o = (unsigned)(sY + 1) * rb + 4u * (unsigned)(x0 - 3 + sX);
#pragma unroll
      for (int i = 0; i < 9; ++i) fs[i] = ldb<float>(Q[i], o);
    }
    asm volatile("; two-step loads issued: interior" ::: "memory");
  } else {
    const char* base = reinterpret_cast<const char*>(src);
    const int xw = wrap(x0 + lx, nx);
#pragma unroll
    for (int k = 0; k < S::KA; ++k)
      if (k * S::WY < S::H1 - (S::WY - 1) || ly + k * S::WY < S::H1)
        pull_rows(base, xw, wrap(y0 - 3 + ly + k * S::WY, ny), nx, ny, fa[k]);
    if (side) pull_rows(base, wrap(x0 - 3 + sX, nx), wrap(y0 - 3 + sY, ny), nx, ny, fs);
    asm volatile("; two-step loads issued: edge" ::: "memory");
  }
  float ra[S::KA], rs = 0.f;
#pragma unroll
  for (int k = 0; k < S::KA; ++k) {
    const int Y = ly + k * S::WY;
    if (Y < S::H1) {
      ra[k] = density(fa[k]);
      s1[Y * S::W1 + lx + 3] = ra[k];
    }
  }
  if (side) {
    rs = density(fs);
    s1[sY * S::W1 + sX] = rs;
  }
  __syncthreads();
  // (B) step t on the tile and a two-node ring (Y in [1, H1 - 1), X in [1, W1 - 1))
#pragma unroll
  for (int k = 0; k < S::KA; ++k) {
    const int Y = ly + k * S::WY;
    if (Y >= 1 && Y < S::H1 - 1) {
      float gx, gy;
      stencil_at<S::W1>(s1, Y * S::W1 + lx + 3, gx, gy);
      collide_node<float>(fa[k], ra[k], gx, gy, c);
      push_node<S, false>(fa[k], lx + 3, Y, sg);
    }
  }
  if (side && sc >= 1 && sc <= 4 && sY >= 1 && sY < S::H1 - 1) {
    float gx, gy;
    stencil_at<S::W1>(s1, sY * S::W1 + sX, gx, gy);
    collide_node<float>(fs, rs, gx, gy, c);
    push_node<S, true>(fs, sX, sY, sg);
  }
  __syncthreads();
  // (C) densities at t + 1 of the tile (own nodes, kept in registers) and its ring
  float fd[S::KD][9], rd[S::KD];
  float* const s2 = s1;
#pragma unroll
  for (int k = 0; k < S::KD; ++k) {
    const int pos = (ly + k * S::WY + 1) * S::LW + lx + 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) fd[k][i] = sg[i * S::G + pos];
    rd[k] = density(fd[k]);
    s2[pos] = rd[k];  // the densities of step t are no longer read (barrier above)
  }
  if (tid < S::NRING) {
    int hx, hy;
    ring_slot<S>(tid, hx, hy);
    const int pos = hy * S::LW + hx;
    float fr[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fr[i] = sg[i * S::G + pos];
    s2[pos] = density(fr);
  }
  __syncthreads();
  // (D) step t + 1 on the tile; with kMid first the state of t + 1, f-bar_i
  // of each tile node, which LDS holds where it streamed to
  const int x = x0 + lx;
  if (x >= nx) return;
  char* const ob = reinterpret_cast<char*>(dst) + (size_t)y0 * rowb;
  char* const mb = kMid ? reinterpret_cast<char*>(mid) + (size_t)y0 * rowb : nullptr;
#pragma unroll
  for (int k = 0; k < S::KD; ++k) {
    const int r = ly + k * S::WY;
    if (y0 + r >= ny) break;
    if constexpr (kMid) {
      const int pos = (r + 1) * S::LW + lx + 1;
      const unsigned o = (unsigned)r * rb + 4u * (unsigned)x;
#pragma unroll
      for (int i = 0; i < 9; ++i)
        __builtin_nontemporal_store(sg[i * S::G + pos + kCy[i] * S::LW + kCx[i]], reinterpret_cast<float*>(mb + i * pb + o));
    }
    float gx, gy;
    stencil_at<S::LW>(s2, (r + 1) * S::LW + lx + 1, gx, gy);
    collide_node<float>(fd[k], rd[k], gx, gy, c);
    const unsigned o = (unsigned)r * rb + 4u * (unsigned)x;
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(fd[k][i], reinterpret_cast<float*>(ob + i * pb + o));
  }
}

// Deterministic FP64 sum of three per-thread values over a block, into this
// block's slot partials[3 b .. 3 b + 2] (added to it if kAdd, else stored):
// a fixed shuffle tree inside each wave, then the waves' sums in wave order.
// red holds 3 doubles per wave of LDS; it may alias LDS the block read
// before the call.
template <class S, bool kAdd>
__device__ __forceinline__ void block_sum3(const double* in, double* red, double* __restrict__ partials) {
  constexpr int NW = S::NTHREADS / 64;
  const int tid = threadIdx.y * S::TX + threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v[3] = {in[0], in[1], in[2]};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += __shfl_down(v[k], off, 64);
  __syncthreads();  // red may alias LDS read above
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) red[k * NW + wave] = v[k];
  __syncthreads();
  if (tid < 3) {
    double s = red[tid * NW];
    for (int w = 1; w < NW; ++w) s += red[tid * NW + w];
    if constexpr (kAdd)
      partials[(size_t)blockIdx.x * 3 + tid] += s;
    else
      partials[(size_t)blockIdx.x * 3 + tid] = s;
  }
}

// Moments: rho and u of main Eq. 5 plus per-workgroup FP64 partial sums of
// mass and lattice momentum (reduced in a fixed order).
template <class St, bool kWideAddr = false>
__global__ __launch_bounds__(MomTile::NTHREADS) void moments_kernel(
    const void* __restrict__ src, const uint16_t* __restrict__ ref_in, float* __restrict__ rho_out,
    float* __restrict__ ux_out, float* __restrict__ uy_out, double* __restrict__ partials, int nx, int ny, int ntx,
    Coef<float> c, RefPoly<float> q) {
  using S = MomTile;
  __shared__ float srho[S::LDS];
  __shared__ double sred[3 * (S::NTHREADS / 64)];
  const size_t N = state_layout(nx, ny, St::ES).ps;
  const int x0 = (blockIdx.x % ntx) * S::TX, y0 = (blockIdx.x / ntx) * S::TY;
  float f[S::NPT][9];
  float rho[S::NPT];
  {
    TileRegs<S, St> R;
    issue_tile<S, St, false, kWideAddr>(planes<typename St::E>(src, N), ref_in, nx, ny, x0, y0, 0, R);
    stage_tile<S, St>(R, q, f, rho, srho, nullptr);
  }
  __syncthreads();
  const int x = x0 + threadIdx.x;
  double sm = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    const int ly = threadIdx.y + k * S::WY, y = y0 + ly;
    if (x >= nx || y >= ny) continue;
    float m[9];
    forward_moments(f[k], m);
    float nb[9], gx, gy;
    neighbours<S>(srho, threadIdx.x + 1, ly + 1, nb);
    stencil(nb[1], nb[2], nb[3], nb[4], nb[5], nb[6], nb[7], nb[8], gx, gy);
    const NodeState<float> s = node_state(m[0], m[3], m[5], gx, gy, c);
    const size_t o = (size_t)y * nx + x;
    if (rho_out) rho_out[o] = m[0];
    if (ux_out) ux_out[o] = s.ux;
    if (uy_out) uy_out[o] = s.uy;
    sm += (double)m[0];
    sx += (double)m[3];
    sy += (double)m[5];
  }
  const double v[3] = {sm, sx, sy};
  block_sum3<S, false>(v, sred, partials);
}

// Sum of the per-workgroup partials in a fixed order: each thread adds a
// strided subset in order, then block_sum3 over the 256 threads.
constexpr int RED = 256;
struct FlatBlock {
  static constexpr int TX = RED, NTHREADS = RED;
};
__global__ __launch_bounds__(RED) void finish_sums(const double* __restrict__ partials, int nblocks,
                                                   double* __restrict__ out) {
  __shared__ double red[3 * (RED / 64)];
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += RED)
    for (int k = 0; k < 3; ++k) a[k] += partials[(size_t)b * 3 + k];
  block_sum3<FlatBlock, false>(a, red, out);  // one block: its slot is out[0..2]
}

// Store the post-streaming populations f of node (x, y) into the pull
// layout: f_i goes to slot (i, x - e_i), encoded against the reference
// density of (x, y), which is also written (2-byte storages).
template <class St>
__device__ __forceinline__ void put_node(int x, int y, int nx, int ny, const float* f, const RefPoly<float>& q,
                                         void* dst, uint16_t* ref_out) {
  using E = typename St::E;
  const Layout L = state_layout(nx, ny, St::ES);
  float rd[9];
  if constexpr (St::kRef) {
    const float r = ref_density(density(f));
    ref_out[(size_t)y * nx + x] = f32_to_f16(r);
#pragma unroll
    for (int i = 0; i < 9; ++i) rd[i] = r;
  }
  E out[9];
  encode<St>(f, rd, q, out);
  E* d = reinterpret_cast<E*>(dst);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int xs = wrap(x - kCx[i], nx), ys = wrap(y - kCy[i], ny);
    d[(size_t)i * L.ps + (size_t)ys * L.rp + xs] = out[i];
  }
}

// Initial state: f^eq(rho0, u0, eta(rho0)) at every node.  Raises *flag on a
// density outside (0, 4/b) or a non-finite input.
constexpr int BLK = 256;
template <class St>
__global__ __launch_bounds__(BLK) void init_kernel(const float* __restrict__ rho0, const float* __restrict__ ux0,
                                                   const float* __restrict__ uy0, void* __restrict__ dst,
                                                   uint16_t* __restrict__ ref_out, int nx, int ny, Coef<float> c,
                                                   RefPoly<float> q, int* flag) {
  const size_t N = (size_t)nx * ny;
  const size_t o = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (o >= N) return;
  const float r = rho0[o], ux = ux0 ? ux0[o] : 0.0f, uy = uy0 ? uy0[o] : 0.0f;
  if (!(r > 0.0f && c.b4 * r < 1.0f) || !isfinite(ux) || !isfinite(uy)) atomicOr(flag, 1);
  float f[9];
  equilibrium_node(r, ux, uy, c, f);
  put_node<St>((int)(o % nx), (int)(o / nx), nx, ny, f, q, dst, ref_out);
}

// Load a post-streaming state.
template <class St>
__global__ __launch_bounds__(BLK) void set_state_kernel(const float* __restrict__ fin, void* __restrict__ dst,
                                                        uint16_t* __restrict__ ref_out, int nx, int ny,
                                                        RefPoly<float> q) {
  const size_t N = (size_t)nx * ny;
  const size_t o = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (o >= N) return;
  float f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = fin[(size_t)i * N + o];
  put_node<St>((int)(o % nx), (int)(o / nx), nx, ny, f, q, dst, ref_out);
}

// Export the post-streaming state f(t).
template <class St>
__global__ __launch_bounds__(BLK) void get_state_kernel(const void* __restrict__ src,
                                                        const uint16_t* __restrict__ ref_in, float* __restrict__ fout,
                                                        int nx, int ny, RefPoly<float> q) {
  using E = typename St::E;
  const size_t N = (size_t)nx * ny;
  const size_t o = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (o >= N) return;
  const int x = (int)(o % nx), y = (int)(o / nx);
  E raw[9];
  const Layout L = state_layout(nx, ny, St::ES);
  if constexpr (!St::kRef) {
    if (wide_state(nx, ny, St::ES)) {
      pull_rows(static_cast<const char*>(src), x, y, nx, ny, raw);
    } else {
      pull_raw<E>(planes<E>(src, L.ps), node_addr<St::ES>(x, y, nx, ny, L.rp), raw);
    }
  } else {
    pull_raw<E>(planes<E>(src, L.ps), node_addr<St::ES>(x, y, nx, ny, L.rp), raw);
  }
  float f[9];
  decode<St>(raw, St::kRef ? ref_in[o] : 0, q, f);
#pragma unroll
  for (int i = 0; i < 9; ++i) fout[(size_t)i * N + o] = f[i];
}

// ---------------------------------------------------------------------------
// Adjoint (reverse mode) of the FP32 step
//
// The adjoint of time t is Lambda_i(x) = dL/d f_i(x, t) for the post-
// streaming populations.  It is kept as eleven planes {L_0..L_8, A_x, A_y}:
//   Lambda_i(x) = L_i(x) + nu(x),   nu(z) = sum_j w_j e_j . A(z - e_j),
// where A(y) = dL/d g(y) for the stencil gradient g of main Eq. 12 at y and
// nu(z) is dL/d rho(z) through the eight stencils that read rho(z).  Keeping
// A instead of adding nu to all nine planes saves a second sweep: the next
// adjoint step forms nu on its tile from a two-node halo of A.
//
// One adjoint step, for every node y (forward state of time t, adjoint of
// time t+1):
//   lam-bar_i(y) = Lambda_i(y + e_i, t+1)   (streaming moved f-bar_i(y) to y + e_i)
//   (L_i(y), A(y), dtheta) = transposed Jacobian of the collision at y
//                            (rho and g recomputed as the forward step has them)
// ---------------------------------------------------------------------------
#ifndef LBM_ADJ_TILE
#define LBM_ADJ_TILE 64, 8, 4
#endif
using AdjTile = TileShape<LBM_ADJ_TILE>;

template <class S>
struct AdjLds {
  static constexpr int AW = S::TX + 4, AH = S::TY + 4, NA = AW * AH;
  static constexpr int NRED = 3 * (S::NTHREADS / 64);  // doubles of the block reduction (one per wave)
  // floats of the LDS buffer that holds the A halo, then the reduction
  static constexpr int NSA = 2 * NA > 2 * NRED ? 2 * NA : 2 * NRED;
};

// A on the tile plus a two-node ring ((TY+4) x (TX+4) nodes), held in
// registers by the thread that stages it: halo node p = tid + r * NTHREADS.
template <class S>
struct AHalo {
  static constexpr int R = (AdjLds<S>::NA + S::NTHREADS - 1) / S::NTHREADS;
  float v[R][2];
};

// Halo coordinates (hx, hy) of the entries p = tid, tid + NTHREADS, ... of
// a W-wide row-major table, stepped without divisions: one division for the
// first entry, then NTHREADS = DY W + DX per step.
template <int W, int NTHREADS>
struct HaloWalk {
  static constexpr int DY = NTHREADS / W, DX = NTHREADS % W;
  int hx, hy;
  __device__ __forceinline__ explicit HaloWalk(int p) : hx(p % W), hy(p / W) {}
  __device__ __forceinline__ void next() {
    hx += DX;
    hy += DY;
    if (hx >= W) hx -= W, ++hy;
  }
};

// 32-bit byte offsets from the A planes' bases: (y rp + x) 4 < 44 nx ny for
// interleaved rows (44 nx ny < 2^32) and < 4 nx ny for planes.
template <class S, bool kInterior = false>
__device__ __forceinline__ void load_a(const float* __restrict__ ax, const float* __restrict__ ay, int nx, int ny,
                                       unsigned rp, int x0, int y0, AHalo<S>& h) {
  using L = AdjLds<S>;
  const int tid = threadIdx.y * S::TX + threadIdx.x;
  HaloWalk<L::AW, S::NTHREADS> w(tid);
#pragma unroll
  for (int r = 0; r < AHalo<S>::R; ++r) {
    const int p = tid + r * S::NTHREADS;
    if (p >= L::NA) break;
    const unsigned yy = kInterior ? (unsigned)(y0 + w.hy - 2) : (unsigned)wrap(y0 + w.hy - 2, ny);
    const unsigned xx = kInterior ? (unsigned)(x0 + w.hx - 2) : (unsigned)wrap(x0 + w.hx - 2, nx);
    const unsigned off = 4u * (yy * rp + xx);
    h.v[r][0] = ldb<float>(reinterpret_cast<const char*>(ax), off);
    h.v[r][1] = ldb<float>(reinterpret_cast<const char*>(ay), off);
    w.next();
  }
}

// The A halo (load_a's registers) into sa[2][AH][AW], a barrier, then nu on
// the tile plus a one-node ring into snu[(TY+2)][LW], and a barrier.
template <class S>
__device__ __forceinline__ void put_nu(const AHalo<S>& h, float* sa, float* snu) {
  using L = AdjLds<S>;
  const int tid = threadIdx.y * S::TX + threadIdx.x;
#pragma unroll
  for (int r = 0; r < AHalo<S>::R; ++r) {
    const int p = tid + r * S::NTHREADS;
    if (p >= L::NA) break;
    sa[p] = h.v[r][0];
    sa[L::NA + p] = h.v[r][1];
  }
  __syncthreads();
  const float third = 1.0f / 3.0f, twelfth = 1.0f / 12.0f;
  const float* sx = sa;
  const float* sy = sa + L::NA;
  HaloWalk<S::LW, S::NTHREADS> w(tid);
  for (int p = tid; p < S::LDS; p += S::NTHREADS, w.next()) {
    const int hx = w.hx, hy = w.hy;
    const int c = (hy + 1) * L::AW + hx + 1;  // the same node in the A halo
    // axis neighbours z - e_j: E -> c-1, W -> c+1, N -> c-AW, S -> c+AW
    const float axis = (sx[c - 1] - sx[c + 1]) + (sy[c - L::AW] - sy[c + L::AW]);
    // diagonals: NE -> c-AW-1 (Ax+Ay), NW -> c-AW+1 (Ay-Ax), SW -> c+AW+1 -(Ax+Ay), SE -> c+AW-1 (Ax-Ay)
    const float diag = (sx[c - L::AW - 1] + sy[c - L::AW - 1]) + (sy[c - L::AW + 1] - sx[c - L::AW + 1]) -
                       (sx[c + L::AW + 1] + sy[c + L::AW + 1]) + (sx[c + L::AW - 1] - sy[c + L::AW - 1]);
    snu[p] = third * axis + twelfth * diag;
  }
  __syncthreads();
}

// nu of the tile plus a one-node ring from the A planes (load_a, put_nu).
template <class S, bool kInterior = false>
__device__ __forceinline__ void stage_nu(const float* __restrict__ ax, const float* __restrict__ ay, int nx, int ny,
                                         unsigned rp, int x0, int y0, float* sa, float* snu) {
  AHalo<S> h;
  load_a<S, kInterior>(ax, ay, nx, ny, rp, x0, y0, h);
  put_nu<S>(h, sa, snu);
}

// Deterministic FP64 block sum of three per-thread FP32 values, added to this
// block's slot of partials (a block always owns the same slot, so sums over
// many launches are reproducible bit for bit).
template <class S>
__device__ __forceinline__ void block_accumulate(const float* th, double* red, double* __restrict__ partials) {
  const double v[3] = {(double)th[0], (double)th[1], (double)th[2]};
  block_sum3<S, true>(v, red, partials);
}

// One tile of the adjoint step (kInterior: interior_tile holds, no wrap).
// Every global load (the forward populations with their ring, the A halo and
// the adjoint populations of the own nodes) is issued before the first
// barrier.
template <class S, bool kInterior, int kMode>
__device__ __forceinline__ void adjoint_tile(const float* __restrict__ fsrc, const float* __restrict__ adj_in,
                                             float* __restrict__ adj_out, int nx, int ny, int x0, int y0,
                                             const Coef<float>& c, float* srho, float* snu, float* sa, float* th) {
  const Layout A = adj_layout(nx, ny);
  const size_t N = A.ps;
  const Planes<float> P = planes<float>(adj_in, N);
  const unsigned rb = 4u * A.rp;
  const int x = x0 + threadIdx.x;
  const unsigned o0 = rb * (unsigned)(y0 + threadIdx.y) + 4u * (unsigned)x;
  float f[S::NPT][9];
  float rho[S::NPT];
  float lb[S::NPT][9];
  AHalo<S> h;
  {
    TileRegs<S, StoreF32> R;
    const Layout Ls = state_layout(nx, ny, 4);
    const int yb = kMode == kBand ? y0 - 2 : 0;  // forward state: rows counted from yb
    if constexpr (kMode == kWide)
      issue_tile<S, StoreF32, false, true>(planes<float>(fsrc, Ls.ps), nullptr, nx, ny, x0, y0, 0, R);
    else
      issue_tile<S, StoreF32, kInterior>(planes<float>(reinterpret_cast<const char*>(fsrc) + (size_t)yb * 4 * Ls.rp, Ls.ps),
                                         nullptr, nx, ny, x0, y0, yb, R);
    load_a<S, kInterior>(adj_in + 9 * N, adj_in + 10 * N, nx, ny, A.rp, x0, y0, h);
    // lam-bar_i(y) = L_i(y + e_i) (+ nu(y + e_i) below)
#pragma unroll
    for (int k = 0; k < S::NPT; ++k) {
      const int y = y0 + threadIdx.y + k * S::WY;
      if (x >= nx || y >= ny) break;
      const unsigned o = o0 + (unsigned)(k * S::WY) * rb;
      if constexpr (kInterior) {
#pragma unroll
        for (int i = 0; i < 9; ++i) lb[k][i] = ldb<float>(P.p[i] + (ptrdiff_t)kCy[i] * rb + kCx[i] * 4, o);
      } else {
        const NodeAddr<4> a = node_addr<4>(x, y, nx, ny, A.rp);
        lb[k][0] = ldb<float>(P.p[0], a.r0 + a.c0);
        lb[k][1] = ldb<float>(P.p[1], a.r0 + a.cp);
        lb[k][2] = ldb<float>(P.p[2], a.rp + a.c0);
        lb[k][3] = ldb<float>(P.p[3], a.r0 + a.cm);
        lb[k][4] = ldb<float>(P.p[4], a.rm + a.c0);
        lb[k][5] = ldb<float>(P.p[5], a.rp + a.cp);
        lb[k][6] = ldb<float>(P.p[6], a.rp + a.cm);
        lb[k][7] = ldb<float>(P.p[7], a.rm + a.cm);
        lb[k][8] = ldb<float>(P.p[8], a.rm + a.cp);
      }
    }
    stage_tile<S, StoreF32>(R, RefPoly<float>{}, f, rho, srho, nullptr);
  }
  put_nu<S>(h, sa, snu);  // its barriers cover srho too
  struct {
    char* p[11];
  } Q;
#pragma unroll
  for (int i = 0; i < 11; ++i) Q.p[i] = reinterpret_cast<char*>(adj_out) + (size_t)i * N * 4;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    const int ly = threadIdx.y + k * S::WY, y = y0 + ly;
    if (x >= nx || y >= ny) break;
    const int hx = threadIdx.x + 1, hy = ly + 1, pos = hy * S::LW + hx;
    float nb[9];
    neighbours<S>(srho, hx, hy, nb);
    float gx, gy;
    stencil(nb[1], nb[2], nb[3], nb[4], nb[5], nb[6], nb[7], nb[8], gx, gy);
#pragma unroll
    for (int i = 0; i < 9; ++i) lb[k][i] += snu[pos + kCy[i] * S::LW + kCx[i]];
    float lf[9], agx = 0.0f, agy = 0.0f;
    collide_node_vjp<float>(f[k], gx, gy, c, lb[k], lf, agx, agy, th);
    const unsigned o = o0 + (unsigned)(k * S::WY) * rb;
    // uniform field bases and one 32-bit lane offset for the eleven stores
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(lf[i], reinterpret_cast<float*>(Q.p[i] + o));
    __builtin_nontemporal_store(agx, reinterpret_cast<float*>(Q.p[9] + o));
    __builtin_nontemporal_store(agy, reinterpret_cast<float*>(Q.p[10] + o));
  }
}

template <class S, int kMode = kAbs>
__global__ __launch_bounds__(S::NTHREADS) void adjoint_step_kernel(const float* __restrict__ fsrc,
                                                                   const float* __restrict__ adj_in,
                                                                   float* __restrict__ adj_out,
                                                                   double* __restrict__ partials, int nx, int ny,
                                                                   int ntx, int ntiles, int strip, Coef<float> c,
                                                                   TileRows rows) {
  using L = AdjLds<S>;
  __shared__ float srho[S::LDS];
  __shared__ float snu[S::LDS];
  __shared__ __align__(8) float sa[L::NSA];
  int tx, ty;
  strip_tile(xcd_tile(blockIdx.x, ntiles), ntx, ntiles / ntx, strip, tx, ty);
  const int x0 = tx * S::TX, y0 = tile_row(rows, ty) * S::TY;
  float th[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (kMode == kWide)  // the tile rows that wrap: never interior
    adjoint_tile<S, false, kWide>(fsrc, adj_in, adj_out, nx, ny, x0, y0, c, srho, snu, sa, th);
  else if (interior_tile<S>(x0, y0, nx, ny))
    adjoint_tile<S, true, kMode>(fsrc, adj_in, adj_out, nx, ny, x0, y0, c, srho, snu, sa, th);
  else
    adjoint_tile<S, false, kMode>(fsrc, adj_in, adj_out, nx, ny, x0, y0, c, srho, snu, sa, th);
  block_accumulate<S>(th, reinterpret_cast<double*>(sa), partials);
}

// Lambda = L + nu on the tile, then either exported (kInit false) or taken
// through the adjoint of the initial equilibrium (kInit true): dL/d rho0 and
// the parameter terms that enter through eta(rho0).
template <class S, bool kInit>
__global__ __launch_bounds__(S::NTHREADS) void adjoint_finish_kernel(
    const float* __restrict__ adj, float* __restrict__ out, const float* __restrict__ rho0,
    const float* __restrict__ ux0, const float* __restrict__ uy0, double* __restrict__ partials, int nx, int ny,
    int ntx, Coef<float> c) {
  using L = AdjLds<S>;
  __shared__ float snu[S::LDS];
  __shared__ __align__(8) float sa[L::NSA];
  const size_t N = (size_t)nx * ny;
  const Layout A = adj_layout(nx, ny);
  const int x0 = (blockIdx.x % ntx) * S::TX, y0 = (blockIdx.x / ntx) * S::TY;
  stage_nu<S>(adj + 9 * A.ps, adj + 10 * A.ps, nx, ny, A.rp, x0, y0, sa, snu);
  float th[3] = {0.0f, 0.0f, 0.0f};
  const int x = x0 + threadIdx.x;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    const int ly = threadIdx.y + k * S::WY, y = y0 + ly;
    if (x >= nx || y >= ny) break;
    const float nu = snu[(ly + 1) * S::LW + threadIdx.x + 1];
    const size_t o = (size_t)y * nx + x, oa = (size_t)y * A.rp + x;
    float lam[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) lam[i] = adj[(size_t)i * A.ps + oa] + nu;
    if constexpr (kInit) {
      out[o] = equilibrium_vjp<float>(rho0[o], ux0 ? ux0[o] : 0.0f, uy0 ? uy0[o] : 0.0f, c, lam, th);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) out[(size_t)i * N + o] = lam[i];
    }
  }
  if constexpr (kInit) block_accumulate<S>(th, reinterpret_cast<double*>(sa), partials);
}

// Adjoint state (adj_layout) from a plain Lambda (planes nx*ny apart):
// L = lam, A = 0.
__global__ __launch_bounds__(BLK) void adjoint_seed_kernel(const float* __restrict__ lam, float* __restrict__ adj,
                                                          int nx, int ny) {
  const size_t N = (size_t)nx * ny;
  const size_t o = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (o >= N) return;
  const Layout A = adj_layout(nx, ny);
  const size_t oa = o / nx * A.rp + o % nx;
#pragma unroll
  for (int i = 0; i < 9; ++i) adj[(size_t)i * A.ps + oa] = lam[(size_t)i * N + o];
  adj[9 * A.ps + oa] = 0.0f;
  adj[10 * A.ps + oa] = 0.0f;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
Coef<float> make_coef(const lbm_derived& d, double varpi, double a, double b) {
  Coef<double> c{};
  const double se = d.s_e, sp = d.s_p, sq = d.s_q, seps = d.s_eps, k = d.k, h = d.h, bs = d.bs;
  c.g2 = d.g2;
  c.kp = d.kp;
  c.rt = d.rt;
  c.a = a;
  c.b4 = 0.25 * b;
  c.kprt = d.kp * d.rt;
  c.e_rho = 0.5 * d.g2 - d.kp * a;
  c.de_rho = d.g2 - 2.0 * d.kp * a;
  c.alpha2 = d.alpha2;
  c.beta2 = d.beta2;
  c.k_seps_h = 0.5 * k * seps;
  c.h_sq_h = 0.5 * h * sq;
  c.b_sq = bs * sq;
  c.b_sq_h = 0.5 * bs * sq;
  c.om_e = 1.0 - 0.5 * se;
  c.om_eps = 1.0 - 0.5 * seps;
  c.om_q = 1.0 - 0.5 * sq;
  c.om_p = 1.0 - 0.5 * sp;
  c.two_om_e = 2.0 - se;
  c.two_om_p = 2.0 - sp;
  c.one_m_seps = 1.0 - seps;
  c.one_m_sq = 1.0 - sq;
  c.cR11 = -(se / (4.0 * varpi)) * (9.0 * (1.0 - k) - 2.0 * (3.0 * k + h));
  c.cR17 = -(3.0 * sp * (2.0 - se)) / (4.0 * (2.0 - sp)) * (9.0 * (1.0 - k) + 2.0 * (3.0 * k + h));
  c.cR18 = 12.0 * sp * (2.0 - se) / (2.0 - sp) * (3.0 * k + h);
  c.cT1 = 1.5 * (2.0 - se);
  c.one_mk = 1.0 - k;
  c.twok_h = 2.0 * k + h;
  c.cX1 = 4.5 * (2.0 - se) * (2.0 * k + h);
  c.cT1a = c.cT1 * (1.0 - k);
  c.cT1b = c.cT1 * (2.0 * k + h);
  c.cR71 = -(se * (2.0 - sp)) / (4.0 * varpi * (2.0 - se)) * (3.0 - 4.0 * bs);
  c.cR77 = -(3.0 * sp / 4.0) * (3.0 + 4.0 * bs);
  c.cT7 = 0.5 * (2.0 - sp);
  c.two_b = 2.0 * bs;
  c.cX7 = -3.0 * (2.0 - sp) * bs;
  c.cR81 = se * (2.0 - sp) / (varpi * (2.0 - se)) * bs;
  c.cR88 = 6.0 * sp * bs;
  c.cT8 = -0.5 * (2.0 - sp) * bs;
  c.cX8 = 1.5 * (2.0 - sp) * bs;
  c.s_e = se;
  c.kq2 = k * (0.5 * se - 1.0) * seps;
  c.s_eps = seps;
  c.s_p = sp;
  c.q1 = (se - c.kq2) * 0.5 * d.g2;
  c.q7 = sp * d.g2 / 12.0;
  c.q2 = seps * 0.5 * d.g2;
  c.s_q = sq;
  c.w_r11 = -c.cR11 / 36.0, c.w_r17 = -c.cR17 / 36.0, c.w_r18 = -c.cR18 / 36.0;
  c.w_t1a = -c.cT1a / 36.0, c.w_x1 = -c.cX1 / 36.0, c.w_t1b = c.cT1b / 36.0, c.w_q1 = c.q1 / 36.0;
  c.w_seps = seps / 36.0, c.w_q2 = c.q2 / 36.0, c.w_sq = sq / 12.0;
  c.w_r71 = -c.cR71 / 4.0, c.w_r77 = -c.cR77 / 4.0, c.w_t7 = -c.cT7 / 4.0, c.w_x7 = -c.cX7 / 4.0;
  c.w_t7b = -c.cT7 * c.two_b / 4.0, c.w_q7 = c.q7 / 4.0;
  c.w_r81 = -c.cR81 / 4.0, c.w_r88 = -c.cR88 / 4.0, c.w_x8 = -c.cX8 / 4.0, c.w_t8 = -c.cT8 / 4.0;
  Coef<float> f;
  const double* src = reinterpret_cast<const double*>(&c);
  float* dstp = reinterpret_cast<float*>(&f);
  static_assert(sizeof(Coef<double>) == 2 * sizeof(Coef<float>), "Coef layout");
  for (size_t i = 0; i < sizeof(Coef<float>) / sizeof(float); ++i) dstp[i] = (float)src[i];
  return f;
}

// Reference populations of the 2-byte storages.  eta(rho) of the model
// (p_LBE = (rho + eta)/3 with the CS pressure) is replaced by its cubic
// least-squares fit on [0, 1.25 rho_l]; any smooth fit keeps encoder and
// decoder consistent, a closer one keeps the stored deviations small.  The
// class values are those of the rest equilibrium:
//   rest  (16 rho + (4 beta2 - 8) eta)/36,  axis rho/9 - (1 + beta2) eta/18,
//   diag  rho/36 + (4 + beta2) eta/36.
RefPoly<float> make_refpoly(const lbm_derived& d, double a, double b, int storage) {
  const int n = 257;
  const double rmax = 1.25 * d.rho_l;
  double A[4][4] = {}, B[4] = {};
  for (int j = 0; j < n; ++j) {
    const double r = rmax * 0.5 * (1.0 - std::cos(M_PI * j / (n - 1)));
    const double v = 0.25 * b * r, w = 1.0 - v;
    const double z = (1.0 + v + v * v - v * v * v) / (w * w * w);
    const double p = d.kp * (r * d.rt * z - a * r * r) + 0.5 * d.g2 * r * r;
    const double eta = 3.0 * p - r;
    const double bas[4] = {1.0, r, r * r, r * r * r};
    for (int u = 0; u < 4; ++u) {
      B[u] += bas[u] * eta;
      for (int v2 = 0; v2 < 4; ++v2) A[u][v2] += bas[u] * bas[v2];
    }
  }
  // Gaussian elimination with partial pivoting (4x4)
  double e[4];
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
    for (int u = 0; u < 4; ++u) std::swap(A[col][u], A[piv][u]);
    std::swap(B[col], B[piv]);
    for (int r = col + 1; r < 4; ++r) {
      const double fac = A[r][col] / A[col][col];
      for (int u = col; u < 4; ++u) A[r][u] -= fac * A[col][u];
      B[r] -= fac * B[col];
    }
  }
  for (int r = 3; r >= 0; --r) {
    double s = B[r];
    for (int u = r + 1; u < 4; ++u) s -= A[r][u] * e[u];
    e[r] = s / A[r][r];
  }
  const double be = d.beta2;
  const double lin[3] = {16.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0};  // coefficient of rho
  const double eta_c[3] = {(4.0 * be - 8.0) / 36.0, -(1.0 + be) / 18.0, (4.0 + be) / 36.0};
  RefPoly<float> q{};
  for (int cls = 0; cls < 3; ++cls)
    for (int u = 0; u < 4; ++u) q.c[cls][u] = (float)(eta_c[cls] * e[u] + (u == 1 ? lin[cls] : 0.0));
  const double S = storage == LBM_FP16 ? 4096.0 : 1.0;
  q.scale = (float)S;
  q.inv_scale = (float)(1.0 / S);
  return q;
}

}  // namespace
}  // namespace lbm

// Scratch of lbm_moments_noalloc: the per-workgroup FP64 partial sums of the
// moments kernel, in a fixed device array instead of memory the library
// allocates (callers that cannot allocate).  Every device holds its own copy
// until the process ends; host code uses the device address taken by
// hipGetSymbolAddress, never this name.  Calls on one device share it.
constexpr size_t kNoallocScratchDoubles = 262144;  // 2 MiB: 87381 workgroups of 64 x 16 nodes
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace lbm {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices];  // address of `scratch` on each device, once taken

// Address of the static scratch on `device`, which must be the current
// device; taken once per device.  nullptr if the runtime cannot give it.
double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_dev[device] = static_cast<double*>(p);
  }
  return g_scratch_dev[device];
}
}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_ctx {
  lbm_params p;
  lbm_derived d;
  Coef<float> c;
  RefPoly<float> q;
  void* buf[2];
  uint16_t* ref[2];  // reference-density planes (2-byte storages)
  int cur;           // buffer holding the pull source of the next step
  bool ready;        // state initialised
  int64_t t;
  hipStream_t stream;
  int device;
  int cus;           // compute units of the device (tile-shape choice)
  int nblocks;       // workgroups of the moments tile grid
  double* scratch;   // nblocks*3 partials, then 3 totals
  int* flag;
  int adj_blocks;    // workgroups of the adjoint tile grid
  double* theta;     // adj_blocks*3 accumulated partials of dL/dtheta, then 3 totals
  double* noalloc;   // the static scratch on this device (lbm_moments_noalloc), or nullptr
};

namespace {

template <class S>
int tiles_x(int nx) { return (nx + S::TX - 1) / S::TX; }

// Tile columns per strip of the tile order (strip_tile) for tiles tx nodes
// wide on a lattice nx nodes wide.  Measured on MI355X for the FP32 step and
// the adjoint, which stream their bytes from HBM: raster order up to 2048
// nodes, beyond that strips a quarter of the lattice wide and at least 1024
// nodes (4096^2: 1024-node strips, +5 %; 16384 x 8192: 4096-node strips,
// +13 % over raster).  The 2-byte steps, bound by the vector ALU, keep
// raster order (one strip).
int strip_width(int nx, int tx, bool raster) {
  const int ntx = (nx + tx - 1) / tx;
  if (raster || nx <= 2048) return ntx;
  const int nodes = nx / 4 < 1024 ? 1024 : nx / 4;
  const int w = nodes / tx;
  return w < 1 ? 1 : (w > ntx ? ntx : w);
}
template <class S>
int tiles_total(int nx, int ny) { return tiles_x<S>(nx) * ((ny + S::TY - 1) / S::TY); }

// Tile rows [lo, hi) whose reads stay inside the lattice (t TY >= 2 and
// t TY + TY + 2 <= ny): the kBand launch of a wide state.
template <class S>
void band_rows(int ny, int& lo, int& hi) {
  lo = (2 + S::TY - 1) / S::TY;
  hi = ny >= S::TY + 2 ? (ny - S::TY - 2) / S::TY + 1 : 0;
  if (hi < lo) hi = lo;
}

// Launch fn(mode, rows, nrows) over every tile row of a lattice: one kAbs
// launch, or for a wide FP32 state a kBand launch over the band rows and a
// kWide launch over the rows at both ends.
template <class S, bool kFP32, class Fn>
void for_tile_rows(int nx, int ny, Fn&& fn) {
  const int nty = (ny + S::TY - 1) / S::TY;
  if constexpr (kFP32) {
    if (wide_state(nx, ny, 4)) {
      // a band of TY + 4 rows must fit 32-bit offsets (lattices up to about
      // 9M nodes wide); wider ones take 64-bit addresses on every tile row
      if (36ull * (unsigned long long)nx * (S::TY + 4) >= (1ull << 32)) {
        fn(std::integral_constant<int, kWide>{}, TileRows{0, nty, 0}, nty);
        return;
      }
      int lo, hi;
      band_rows<S>(ny, lo, hi);
      if (hi > lo) fn(std::integral_constant<int, kBand>{}, TileRows{lo, hi - lo, 0}, hi - lo);
      fn(std::integral_constant<int, kWide>{}, TileRows{0, lo, hi}, lo + nty - hi);
      return;
    }
  }
  fn(std::integral_constant<int, kAbs>{}, TileRows{0, nty, 0}, nty);
}

// One step of storage St with tile shape S from the buffer src (and its
// reference plane) to dst, on the context's stream.
template <class St, class S>
void launch_step_tiles(const lbm_ctx* ctx, const void* src, void* dst, const uint16_t* ref_in, uint16_t* ref_out) {
  const int nx = ctx->p.nx, ny = ctx->p.ny, ntx = tiles_x<S>(nx);
  for_tile_rows<S, !St::kRef>(nx, ny, [&](auto mode, TileRows rows, int nrows) {
    step_kernel<S, St, decltype(mode)::value><<<ntx * nrows, dim3(S::TX, S::WY), 0, ctx->stream>>>(
        src, dst, ref_in, ref_out, nx, ny, ntx, ntx * nrows, strip_width(nx, S::TX, St::kRef), ctx->c, ctx->q,
        rows);
  });
}

// Smaller tiles for small lattices: the storage's own tile while it gives at
// least one tile per CU, then 128 x 8 (FP32), then 64 x 4.  Measured, FP32
// step: 256^2 6.0 / 4.8 / 3.6 us (256 x 8 / 128 x 8 / 64 x 4), 512^2 7.4 /
// 5.9 / 6.1 us, 1024^2 19.4 / 20.2 / 21.0 us.  The per-node arithmetic does
// not depend on the tile, so every choice gives the same bits.
using SmallTile = TileShape<64, 4, 4>;
using MidTileF32 = TileShape<128, 8, 4>;

template <class St>
void launch_step(const lbm_ctx* ctx, const void* src, void* dst, const uint16_t* ref_in, uint16_t* ref_out) {
  const int nx = ctx->p.nx, ny = ctx->p.ny;
  if (tiles_total<StepTile<St>>(nx, ny) >= ctx->cus) return launch_step_tiles<St, StepTile<St>>(ctx, src, dst, ref_in, ref_out);
  if constexpr (std::is_same_v<St, StoreF32>)
    if (tiles_total<MidTileF32>(nx, ny) >= ctx->cus)
      return launch_step_tiles<St, MidTileF32>(ctx, src, dst, ref_in, ref_out);
  launch_step_tiles<St, SmallTile>(ctx, src, dst, ref_in, ref_out);
}

// Two FP32 steps per launch (step2_kernel) on the largest of three tiles
// that gives at least one tile per CU: 64 x 24, else 64 x 16, else 32 x 8.
// On the small lattices of the last two a step lasts a few microseconds and
// the launches set the pace, so half the launches outweigh the larger share
// of recomputed ring nodes.  Measured, time per step against single steps:
// 256^2 2.92 against 3.61 us (32 x 8; 64 x 16: 3.93), 512^2 4.14 against
// 5.37 us (64 x 16; 32 x 8: 4.68); 32 x 16 and 64 x 8 were no faster.  The
// tiles address TY + 8 rows of 36 nx bytes from one base with 32-bit
// offsets, which bounds the width (about 3.7M nodes); wider lattices take
// single steps.
#ifndef LBM_FUSE_STEPS
#define LBM_FUSE_STEPS 1
#endif
using Step2Mid = Tile2Shape<64, 16, 8>;
using Step2Small = Tile2Shape<32, 8, 8>;
static_assert(Step2Mid::TY <= Step2Tile::TY && Step2Small::TY <= Step2Tile::TY,
              "the width bound of the large tile covers the others");

// 0: single steps; 1, 2, 3: two steps on Step2Tile, Step2Mid, Step2Small.
int step2_shape(const lbm_ctx* ctx) {
  const int nx = ctx->p.nx, ny = ctx->p.ny;
  const unsigned long long band = 36ull * (unsigned long long)nx * (Step2Tile::TY + 8);
  if (!LBM_FUSE_STEPS || ctx->p.storage != LBM_FP32 || band >= (1ull << 32)) return 0;
  if (tiles_total<Step2Tile>(nx, ny) >= ctx->cus) return 1;
  return tiles_total<Step2Mid>(nx, ny) >= ctx->cus ? 2 : 3;
}
bool use_step2(const lbm_ctx* ctx) { return step2_shape(ctx) != 0; }

// src (time t) -> dst (time t + 2), and mid (time t + 1) if kMid.
template <class S, bool kMid>
void launch_step2_on(const lbm_ctx* ctx, const void* src, void* mid, void* dst) {
  const int nx = ctx->p.nx, ny = ctx->p.ny, ntx = tiles_x<S>(nx), nt = tiles_total<S>(nx, ny);
  step2_kernel<S, kMid><<<nt, dim3(S::TX, S::WY), 0, ctx->stream>>>(
      static_cast<const float*>(src), static_cast<float*>(mid), static_cast<float*>(dst), nx, ny, ntx, nt,
      strip_width(nx, S::TX, false), ctx->c);
}
template <bool kMid>
void launch_step2(const lbm_ctx* ctx, const void* src, void* mid, void* dst) {
  switch (step2_shape(ctx)) {
    case 1: launch_step2_on<Step2Tile, kMid>(ctx, src, mid, dst); break;
    case 2: launch_step2_on<Step2Mid, kMid>(ctx, src, mid, dst); break;
    default: launch_step2_on<Step2Small, kMid>(ctx, src, mid, dst); break;
  }
}

int check_ctx(const lbm_ctx* ctx, bool need_state) {
  if (!ctx) return fail(LBM_EINVAL, "context is NULL");
  if (need_state && !ctx->ready) return fail(LBM_ESTATE, "state not initialised (call lbm_init or lbm_set_state)");
  return LBM_OK;
}

int set_device(const lbm_ctx* ctx) {
  int cur = -1;
  HIP_OK(hipGetDevice(&cur));
  if (cur != ctx->device) HIP_OK(hipSetDevice(ctx->device));
  return LBM_OK;
}

// Workgroups of one node per thread; lbm_create admits 9 nx ny < 2^31, so
// the count fits a grid dimension.
unsigned grid1(size_t n) { return static_cast<unsigned>((n + BLK - 1) / BLK); }

// Call fn with the storage policy of the context.
template <class Fn>
int with_storage(const lbm_ctx* ctx, Fn&& fn) {
  switch (ctx->p.storage) {
    case LBM_FP32: return fn(StoreF32{});
    case LBM_FP16: return fn(Store16<LBM_FP16>{});
    default: return fn(Store16<LBM_BF16>{});
  }
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err; }

int lbm_derive(const lbm_params* p, lbm_derived* out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  return lbm::derive(p, out, g_err, sizeof g_err);
}

int lbm_sigma_paper(double width, double tr, double a, double b, double r_gas, double* sigma_out) {
  if (!sigma_out) return fail(LBM_EINVAL, "sigma_out is NULL");
  if (!(width > 0) || !(tr > 0 && tr < 1) || !(a > 0) || !(b > 0) || !(r_gas > 0))
    return fail(LBM_EINVAL, "invalid parameter: width, a, b, r_gas > 0 and 0 < tr < 1 required");
  int st = lbm::sigma_paper(width, tr, a, b, r_gas, sigma_out);
  return st ? fail(st, "no two-phase coexistence found at tr = %g", tr) : LBM_OK;
}

size_t lbm_state_bytes(const lbm_params* p) {
  char msg[256];
  if (lbm::validate(p, msg, sizeof msg)) return 0;
  const int es = p->storage == LBM_FP32 ? 4 : 2;
  return (size_t)9 * plane_elems(p->nx, p->ny, es) * es;
}

size_t lbm_ref_bytes(const lbm_params* p) {
  char msg[256];
  if (lbm::validate(p, msg, sizeof msg) || p->storage == LBM_FP32) return 0;
  return (size_t)2 * p->nx * p->ny * 2;
}

int lbm_create(lbm_ctx** out, const lbm_params* p, void* f_a, void* f_b, void* rho_ref, void* stream) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_derived d;
  int st = lbm::derive(p, &d, g_err, sizeof g_err);
  if (st) return st;
  if (!f_a || !f_b || f_a == f_b) return fail(LBM_EINVAL, "f_a and f_b must be two distinct device buffers");
  if (p->storage != LBM_FP32 && !rho_ref)
    return fail(LBM_EINVAL, "the 2-byte storages need the reference-density buffer rho_ref");
  lbm_ctx* c = new (std::nothrow) lbm_ctx{};
  if (!c) return fail(LBM_EHIP, "out of host memory");
  c->p = *p;
  c->d = d;
  c->c = make_coef(d, p->varpi, p->a, p->b);
  c->q = make_refpoly(d, p->a, p->b, p->storage);
  c->buf[0] = f_a;
  c->buf[1] = f_b;
  const size_t N = (size_t)p->nx * p->ny;
  c->ref[0] = p->storage == LBM_FP32 ? nullptr : reinterpret_cast<uint16_t*>(rho_ref);
  c->ref[1] = p->storage == LBM_FP32 ? nullptr : reinterpret_cast<uint16_t*>(rho_ref) + N;
  c->cur = 0;
  c->ready = false;
  c->t = 0;
  c->stream = (hipStream_t)stream;
  c->nblocks = tiles_total<MomTile>(p->nx, p->ny);
  c->adj_blocks = p->storage == LBM_FP32 ? tiles_total<AdjTile>(p->nx, p->ny) : 0;
  const size_t mom_doubles = 3 * (size_t)c->nblocks + 3 + 8;  // + the status word
  const size_t th_doubles = 3 * (size_t)c->adj_blocks + 3;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e == hipSuccess) e = hipMalloc(&c->scratch, sizeof(double) * (mom_doubles + th_doubles));
  if (e == hipSuccess) e = hipMemsetAsync(c->scratch, 0, sizeof(double) * (mom_doubles + th_doubles), c->stream);
  if (e != hipSuccess) {
    if (c->scratch) (void)hipFree(c->scratch);
    delete c;
    return fail(LBM_EHIP, "lbm_create: %s", hipGetErrorString(e));
  }
  c->flag = reinterpret_cast<int*>(c->scratch + 3 * (size_t)c->nblocks + 3);
  c->theta = c->scratch + mom_doubles;
  c->noalloc = noalloc_scratch(c->device);  // c->device is current here
  *out = c;
  return LBM_OK;
}

int lbm_set_stream(lbm_ctx* ctx, void* stream) {
  if (int st = check_ctx(ctx, false)) return st;
  const hipStream_t next = (hipStream_t)stream;
  if (next != ctx->stream) {
    // work queued on the old stream precedes everything issued on the new one
    if (int st = set_device(ctx)) return st;
    hipEvent_t ev;
    HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, ctx->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(next, ev, 0);
    (void)hipEventDestroy(ev);  // released once the wait has been satisfied
    if (e != hipSuccess) return fail(LBM_EHIP, "lbm_set_stream: %s", hipGetErrorString(e));
  }
  ctx->stream = next;
  return LBM_OK;
}

int lbm_init(lbm_ctx* ctx, const float* rho0, const float* ux0, const float* uy0) {
  if (int st = check_ctx(ctx, false)) return st;
  if (!rho0) return fail(LBM_EINVAL, "rho0 is NULL");
  if (int st = set_device(ctx)) return st;
  const size_t N = (size_t)ctx->p.nx * ctx->p.ny;
  HIP_OK(hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream));
  int st = with_storage(ctx, [&](auto store) -> int {
    using St = decltype(store);
    init_kernel<St><<<grid1(N), BLK, 0, ctx->stream>>>(rho0, ux0, uy0, ctx->buf[0], ctx->ref[0], ctx->p.nx,
                                                        ctx->p.ny, ctx->c, ctx->q, ctx->flag);
    HIP_OK(hipGetLastError());
    return LBM_OK;
  });
  if (st) return st;
  int flag = 0;
  HIP_OK(hipMemcpyAsync(&flag, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  if (flag) {
    ctx->ready = false;
    return fail(LBM_EINVAL, "rho0 must be finite and in (0, 4/b), u0 finite");
  }
  ctx->cur = 0;
  ctx->t = 0;
  ctx->ready = true;
  return LBM_OK;
}

int lbm_set_state(lbm_ctx* ctx, const float* f) {
  if (int st = check_ctx(ctx, false)) return st;
  if (!f) return fail(LBM_EINVAL, "f is NULL");
  if (int st = set_device(ctx)) return st;
  const size_t N = (size_t)ctx->p.nx * ctx->p.ny;
  int st = with_storage(ctx, [&](auto store) -> int {
    using St = decltype(store);
    set_state_kernel<St><<<grid1(N), BLK, 0, ctx->stream>>>(f, ctx->buf[0], ctx->ref[0], ctx->p.nx, ctx->p.ny,
                                                             ctx->q);
    HIP_OK(hipGetLastError());
    return LBM_OK;
  });
  if (st) return st;
  ctx->cur = 0;
  ctx->t = 0;
  ctx->ready = true;
  return LBM_OK;
}

int lbm_get_state(lbm_ctx* ctx, float* f) {
  if (int st = check_ctx(ctx, true)) return st;
  if (!f) return fail(LBM_EINVAL, "f is NULL");
  if (int st = set_device(ctx)) return st;
  const size_t N = (size_t)ctx->p.nx * ctx->p.ny;
  return with_storage(ctx, [&](auto store) -> int {
    using St = decltype(store);
    get_state_kernel<St><<<grid1(N), BLK, 0, ctx->stream>>>(ctx->buf[ctx->cur], ctx->ref[ctx->cur], f, ctx->p.nx,
                                                             ctx->p.ny, ctx->q);
    HIP_OK(hipGetLastError());
    return LBM_OK;
  });
}

int lbm_step(lbm_ctx* ctx, int32_t n) {
  if (int st = check_ctx(ctx, true)) return st;
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  if (int st = set_device(ctx)) return st;
  int st = with_storage(ctx, [&](auto store) -> int {
    using St = decltype(store);
    for (int32_t s = 0; s < n;) {
      const int a = ctx->cur, b = ctx->cur ^ 1;
      if (std::is_same_v<St, StoreF32> && n - s >= 2 && use_step2(ctx)) {
        launch_step2<false>(ctx, ctx->buf[a], nullptr, ctx->buf[b]);
        s += 2;
      } else {
        launch_step<St>(ctx, ctx->buf[a], ctx->buf[b], ctx->ref[a], ctx->ref[b]);
        ++s;
      }
      ctx->cur = b;
    }
    HIP_OK(hipGetLastError());
    return LBM_OK;
  });
  if (st) return st;
  ctx->t += n;
  return LBM_OK;
}

namespace {
// The moments kernel over the current state, its per-workgroup partials
// into `partials` (3 per workgroup of tiles_total<MomTile>).
int launch_moments(const lbm_ctx* ctx, float* rho, float* ux, float* uy, double* partials) {
  using S = MomTile;
  return with_storage(ctx, [&](auto store) -> int {
    using St = decltype(store);
    auto go = [&](auto wide) {
      moments_kernel<St, decltype(wide)::value><<<tiles_total<S>(ctx->p.nx, ctx->p.ny), dim3(S::TX, S::WY), 0,
                                                  ctx->stream>>>(ctx->buf[ctx->cur], ctx->ref[ctx->cur], rho, ux, uy,
                                                                 partials, ctx->p.nx, ctx->p.ny,
                                                                 tiles_x<S>(ctx->p.nx), ctx->c, ctx->q);
    };
    if constexpr (!St::kRef) {
      if (wide_state(ctx->p.nx, ctx->p.ny, 4))
        go(std::true_type{});
      else
        go(std::false_type{});
    } else {
      go(std::false_type{});
    }
    HIP_OK(hipGetLastError());
    return LBM_OK;
  });
}
}  // namespace

int lbm_moments(lbm_ctx* ctx, float* rho, float* ux, float* uy, double totals[3]) {
  if (int st = check_ctx(ctx, true)) return st;
  if (int st = set_device(ctx)) return st;
  if (int st = launch_moments(ctx, rho, ux, uy, ctx->scratch)) return st;
  if (!totals) return LBM_OK;
  double* tot = ctx->scratch + 3 * (size_t)ctx->nblocks;
  finish_sums<<<1, RED, 0, ctx->stream>>>(ctx->scratch, ctx->nblocks, tot);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(totals, tot, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(totals[k])) return fail(LBM_ENONFINITE, "non-finite total (%d): the state has diverged", k);
  return LBM_OK;
}

int lbm_moments_noalloc(lbm_ctx* ctx, float* rho, float* ux, float* uy, double* totals_dev) {
  if (!ctx) return fail(LBM_EINVAL, "context is NULL");
  if (3 * (size_t)ctx->nblocks > kNoallocScratchDoubles)
    return fail(LBM_EINVAL,
                "lbm_moments_noalloc: a %d x %d lattice needs %zu doubles of scratch, the static maximum is %zu "
                "(%zu workgroups of 64 x 16 nodes); use lbm_moments",
                ctx->p.nx, ctx->p.ny, 3 * (size_t)ctx->nblocks, kNoallocScratchDoubles, kNoallocScratchDoubles / 3);
  if (int st = check_ctx(ctx, true)) return st;
  if (!ctx->noalloc) return fail(LBM_EHIP, "lbm_moments_noalloc: the static scratch has no device address");
  if (int st = set_device(ctx)) return st;
  if (int st = launch_moments(ctx, rho, ux, uy, ctx->noalloc)) return st;
  if (totals_dev) {
    finish_sums<<<1, RED, 0, ctx->stream>>>(ctx->noalloc, ctx->nblocks, totals_dev);
    HIP_OK(hipGetLastError());
  }
  return LBM_OK;
}

size_t lbm_checkpoint_bytes(const lbm_params* p) {
  const size_t s = lbm_state_bytes(p);
  return s == 0 || p->storage == LBM_FP32 ? s : s + (size_t)2 * p->nx * p->ny;
}

int lbm_save_state(lbm_ctx* ctx, void* dst) {
  if (int st = check_ctx(ctx, true)) return st;
  if (!dst) return fail(LBM_EINVAL, "dst is NULL");
  if (int st = set_device(ctx)) return st;
  const size_t sb = lbm_state_bytes(&ctx->p);
  HIP_OK(hipMemcpyAsync(dst, ctx->buf[ctx->cur], sb, hipMemcpyDeviceToDevice, ctx->stream));
  if (ctx->p.storage != LBM_FP32)
    HIP_OK(hipMemcpyAsync(static_cast<char*>(dst) + sb, ctx->ref[ctx->cur], (size_t)2 * ctx->p.nx * ctx->p.ny,
                          hipMemcpyDeviceToDevice, ctx->stream));
  return LBM_OK;
}

int lbm_load_state(lbm_ctx* ctx, const void* src, int64_t t) {
  if (int st = check_ctx(ctx, false)) return st;
  if (!src) return fail(LBM_EINVAL, "src is NULL");
  if (t < 0) return fail(LBM_EINVAL, "t must be >= 0");
  if (int st = set_device(ctx)) return st;
  const size_t sb = lbm_state_bytes(&ctx->p);
  HIP_OK(hipMemcpyAsync(ctx->buf[0], src, sb, hipMemcpyDeviceToDevice, ctx->stream));
  if (ctx->p.storage != LBM_FP32)
    HIP_OK(hipMemcpyAsync(ctx->ref[0], static_cast<const char*>(src) + sb, (size_t)2 * ctx->p.nx * ctx->p.ny,
                          hipMemcpyDeviceToDevice, ctx->stream));
  ctx->cur = 0;
  ctx->t = t;
  ctx->ready = true;
  return LBM_OK;
}

namespace {
int need_fp32(const lbm_ctx* ctx, const char* what) {
  if (ctx->p.storage != LBM_FP32) return fail(LBM_EINVAL, "%s is available for LBM_FP32 storage only", what);
  return LBM_OK;
}
}  // namespace

int lbm_step_saved(lbm_ctx* ctx, const void* src, void* dst) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "lbm_step_saved")) return st;
  if (!src || !dst || src == dst) return fail(LBM_EINVAL, "src and dst must be two distinct device buffers");
  if (int st = set_device(ctx)) return st;
  launch_step<StoreF32>(ctx, src, dst, nullptr, nullptr);
  HIP_OK(hipGetLastError());
  return LBM_OK;
}

int lbm_step_saved_chain(lbm_ctx* ctx, void* const* bufs, int32_t n) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "lbm_step_saved_chain")) return st;
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  if (!bufs) return fail(LBM_EINVAL, "bufs is NULL");
  for (int32_t j = 0; j < n; ++j)
    if (!bufs[j] || !bufs[j + 1] || bufs[j] == bufs[j + 1])
      return fail(LBM_EINVAL, "bufs[%d] and bufs[%d] must be two distinct device buffers", j, j + 1);
  if (int st = set_device(ctx)) return st;
  for (int32_t j = 0; j < n;) {
    // two steps per launch where the state two steps on goes to a third buffer
    if (n - j >= 2 && use_step2(ctx) && bufs[j + 2] != bufs[j]) {
      launch_step2<true>(ctx, bufs[j], bufs[j + 1], bufs[j + 2]);
      j += 2;
    } else {
      launch_step<StoreF32>(ctx, bufs[j], bufs[j + 1], nullptr, nullptr);
      ++j;
    }
  }
  HIP_OK(hipGetLastError());
  return LBM_OK;
}

size_t lbm_adjoint_bytes(const lbm_params* p) {
  char msg[256];
  if (lbm::validate(p, msg, sizeof msg) || p->storage != LBM_FP32) return 0;
  return (size_t)11 * plane_elems(p->nx, p->ny, 4) * sizeof(float);
}

int lbm_adjoint_seed(lbm_ctx* ctx, const float* lam, void* adj) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "the adjoint")) return st;
  if (!lam || !adj) return fail(LBM_EINVAL, "lam and adj must be device buffers");
  if (int st = set_device(ctx)) return st;
  const size_t N = (size_t)ctx->p.nx * ctx->p.ny;
  adjoint_seed_kernel<<<grid1(N), BLK, 0, ctx->stream>>>(lam, static_cast<float*>(adj), ctx->p.nx, ctx->p.ny);
  HIP_OK(hipGetLastError());
  return LBM_OK;
}

// One adjoint step on the context's stream (split like the forward step for
// wide FP32 states).  Blocks of both launches add into the partial-sum
// slots 0 .. grid-1 in launch order, so the sums stay reproducible.
static void launch_adjoint(const lbm_ctx* ctx, const void* f_t, const void* adj_next, void* adj_out) {
  using S = AdjTile;
  const int nx = ctx->p.nx, ny = ctx->p.ny, ntx = tiles_x<S>(nx);
  for_tile_rows<S, true>(nx, ny, [&](auto mode, TileRows rows, int nrows) {
    adjoint_step_kernel<S, decltype(mode)::value><<<ntx * nrows, dim3(S::TX, S::WY), 0, ctx->stream>>>(
        static_cast<const float*>(f_t), static_cast<const float*>(adj_next), static_cast<float*>(adj_out),
        ctx->theta, nx, ny, ntx, ntx * nrows, strip_width(nx, S::TX, false), ctx->c, rows);
  });
}

int lbm_adjoint_step(lbm_ctx* ctx, const void* f_t, const void* adj_next, void* adj_out) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "the adjoint")) return st;
  if (!f_t || !adj_next || !adj_out || adj_next == adj_out)
    return fail(LBM_EINVAL, "f_t, adj_next and adj_out must be device buffers, adj_next != adj_out");
  if (int st = set_device(ctx)) return st;
  launch_adjoint(ctx, f_t, adj_next, adj_out);
  HIP_OK(hipGetLastError());
  return LBM_OK;
}

int lbm_adjoint_run(lbm_ctx* ctx, const void* const* f_states, int32_t n, void* adj_a, void* adj_b,
                    int32_t* which) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "the adjoint")) return st;
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (!which) return fail(LBM_EINVAL, "which is NULL");
  if (!adj_a || !adj_b || adj_a == adj_b) return fail(LBM_EINVAL, "adj_a and adj_b must be two distinct device buffers");
  if (n > 0 && !f_states) return fail(LBM_EINVAL, "f_states is NULL");
  for (int32_t j = 0; j < n; ++j)
    if (!f_states[j]) return fail(LBM_EINVAL, "f_states[%d] is NULL", j);
  if (int st = set_device(ctx)) return st;
  void* buf[2] = {adj_a, adj_b};
  int cur = 0;
  for (int32_t j = n - 1; j >= 0; --j) {
    launch_adjoint(ctx, f_states[j], buf[cur], buf[cur ^ 1]);
    cur ^= 1;
  }
  HIP_OK(hipGetLastError());
  *which = cur;
  return LBM_OK;
}

int lbm_adjoint_get(lbm_ctx* ctx, const void* adj, float* lam) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "the adjoint")) return st;
  if (!adj || !lam) return fail(LBM_EINVAL, "adj and lam must be device buffers");
  if (int st = set_device(ctx)) return st;
  using S = AdjTile;
  adjoint_finish_kernel<S, false><<<ctx->adj_blocks, dim3(S::TX, S::WY), 0, ctx->stream>>>(
      static_cast<const float*>(adj), lam, nullptr, nullptr, nullptr, nullptr, ctx->p.nx, ctx->p.ny,
      tiles_x<S>(ctx->p.nx), ctx->c);
  HIP_OK(hipGetLastError());
  return LBM_OK;
}

int lbm_adjoint_init(lbm_ctx* ctx, const float* rho0, const float* ux0, const float* uy0, const void* adj0,
                     float* drho0) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "the adjoint")) return st;
  if (!rho0 || !adj0 || !drho0) return fail(LBM_EINVAL, "rho0, adj0 and drho0 must be device buffers");
  if (int st = set_device(ctx)) return st;
  using S = AdjTile;
  adjoint_finish_kernel<S, true><<<ctx->adj_blocks, dim3(S::TX, S::WY), 0, ctx->stream>>>(
      static_cast<const float*>(adj0), drho0, rho0, ux0, uy0, ctx->theta, ctx->p.nx, ctx->p.ny,
      tiles_x<S>(ctx->p.nx), ctx->c);
  HIP_OK(hipGetLastError());
  return LBM_OK;
}

int lbm_adjoint_theta(lbm_ctx* ctx, double dtheta[3], int32_t reset) {
  if (int st = check_ctx(ctx, false)) return st;
  if (int st = need_fp32(ctx, "the adjoint")) return st;
  if (int st = set_device(ctx)) return st;
  double* tot = ctx->theta + 3 * (size_t)ctx->adj_blocks;
  if (dtheta) {
    finish_sums<<<1, RED, 0, ctx->stream>>>(ctx->theta, ctx->adj_blocks, tot);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(dtheta, tot, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  }
  if (reset) HIP_OK(hipMemsetAsync(ctx->theta, 0, 3 * sizeof(double) * (size_t)ctx->adj_blocks, ctx->stream));
  if (dtheta) {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(dtheta[k])) return fail(LBM_ENONFINITE, "non-finite parameter gradient (%d)", k);
  }
  return LBM_OK;
}

int lbm_adjoint_params(lbm_ctx* ctx, double dparams[3], double dtheta[3], int32_t reset) {
  if (!dparams) return fail(LBM_EINVAL, "dparams is NULL");
  double th[3];
  if (int st = lbm_adjoint_theta(ctx, th, reset)) return st;
  double jac[9];
  if (int st = lbm::param_jacobian(&ctx->p, jac, g_err, sizeof g_err)) return st;
  for (int j = 0; j < 3; ++j) dparams[j] = jac[j] * th[0] + jac[3 + j] * th[1] + jac[6 + j] * th[2];
  if (dtheta)
    for (int k = 0; k < 3; ++k) dtheta[k] = th[k];
  return LBM_OK;
}

int lbm_param_jacobian(const lbm_params* p, double jac[9]) {
  if (!jac) return fail(LBM_EINVAL, "jac is NULL");
  return lbm::param_jacobian(p, jac, g_err, sizeof g_err);
}

int64_t lbm_time(const lbm_ctx* ctx) { return ctx ? ctx->t : -1; }

int lbm_get_derived(const lbm_ctx* ctx, lbm_derived* out) {
  if (int st = check_ctx(ctx, false)) return st;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = ctx->d;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->scratch) {
    int cur = -1;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != ctx->device;
    if (other) (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->scratch);  // waits for the context's work in flight
    if (other) (void)hipSetDevice(cur);
  }
  delete ctx;
}

}  // extern "C"
