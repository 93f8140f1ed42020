// HIP kernels and C-ABI entry points of the self-tuning-EOS D2Q9 library
// (gfx950).  See include/lbm.h for the contract of every entry point.
//
// Data layout: structure of arrays, population i at offset i*nx*ny, x
// fastest.  Two caller-owned buffers A and B alternate; the buffer that is
// read by the next step holds the post-collision populations of the previous
// step at their source node ("pull" streaming: f_i(x, t) = src_i(x - e_i)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

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
// Index helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Pull the nine populations arriving at node (x, y): f_i(x) = src_i(x - e_i).
// xm/xp, ym/yp are the periodic neighbours x-1/x+1, y-1/y+1.
__device__ __forceinline__ void pull9(const float* __restrict__ src, size_t N, int nx, int x, int xm, int xp,
                                      int y, int ym, int yp, float* f) {
  const size_t r0 = (size_t)y * nx, rm = (size_t)ym * nx, rp = (size_t)yp * nx;
  f[0] = src[r0 + x];
  f[1] = src[1 * N + r0 + xm];
  f[2] = src[2 * N + rm + x];
  f[3] = src[3 * N + r0 + xp];
  f[4] = src[4 * N + rp + x];
  f[5] = src[5 * N + rm + xm];
  f[6] = src[6 * N + rm + xp];
  f[7] = src[7 * N + rp + xp];
  f[8] = src[8 * N + rp + xm];
}

// The same pull with 32-bit byte offsets from per-plane base pointers (the
// bases are uniform, so the loads use a scalar base plus one vector offset).
// A node is addressed by its three row offsets (row * nx * 4 for rows y,
// y-1, y+1) and three column offsets (4 x for x, x-1, x+1).
struct NodeAddr {
  unsigned r0, rm, rp, c0, cm, cp;
};

__device__ __forceinline__ NodeAddr node_addr(int x, int y, int nx, int ny) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const unsigned rb = 4u * (unsigned)nx;
  return {rb * (unsigned)y, rb * (unsigned)ym, rb * (unsigned)yp, 4u * (unsigned)x, 4u * (unsigned)xm,
          4u * (unsigned)xp};
}

__device__ __forceinline__ float ldb(const char* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const float*>(base + off);
}

struct Planes {
  const char* p[9];
};

__device__ __forceinline__ Planes planes(const float* src, size_t N) {
  Planes P;
#pragma unroll
  for (int i = 0; i < 9; ++i) P.p[i] = reinterpret_cast<const char*>(src + (size_t)i * N);
  return P;
}

struct OutPlanes {
  char* p[9];
};

__device__ __forceinline__ OutPlanes out_planes(float* dst, size_t N) {
  OutPlanes P;
#pragma unroll
  for (int i = 0; i < 9; ++i) P.p[i] = reinterpret_cast<char*>(dst + (size_t)i * N);
  return P;
}

__device__ __forceinline__ void pull9b(const Planes& P, const NodeAddr& a, float* f) {
  f[0] = ldb(P.p[0], a.r0 + a.c0);
  f[1] = ldb(P.p[1], a.r0 + a.cm);
  f[2] = ldb(P.p[2], a.rm + a.c0);
  f[3] = ldb(P.p[3], a.r0 + a.cp);
  f[4] = ldb(P.p[4], a.rp + a.c0);
  f[5] = ldb(P.p[5], a.rm + a.cm);
  f[6] = ldb(P.p[6], a.rm + a.cp);
  f[7] = ldb(P.p[7], a.rp + a.cp);
  f[8] = ldb(P.p[8], a.rp + a.cm);
}

// Tile order across the eight XCDs of the chip: workgroups are dealt to the
// XCDs round-robin by dispatch index, so dispatch b runs on XCD b % 8.  Give
// each XCD one contiguous run of tiles (in raster order) so that the tiles
// whose halo lines overlap share that XCD's L2.  A bijection onto
// [0, ntiles) for any ntiles.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int q = ntiles >> 3, r = ntiles & 7, xcd = b & 7, local = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + local;
}

// ---------------------------------------------------------------------------
// Fused step: tile of TX x TY nodes per workgroup of TX x WY threads; each
// thread owns NPT = TY/WY nodes of one column.  The tile plus a one-node
// ring of densities is staged in LDS for the force stencil; ring nodes pull
// their own populations (L2 hits: the neighbouring tiles run on the same XCD).
// ---------------------------------------------------------------------------
template <int TX_, int TY_, int WY_>
struct TileShape {
  static constexpr int TX = TX_, TY = TY_, WY = WY_, NPT = TY / WY, LW = TX + 2;
  static constexpr int NRING = 2 * LW + 2 * TY, NTHREADS = TX * WY, LDS = (TY + 2) * LW;
  static_assert(TY % WY == 0, "rows per thread");
  static_assert(NRING <= NTHREADS, "one ring node per thread");
};

// Tile of the step kernel (TX, TY, WY); a compile-time tuning knob.
#ifndef LBM_STEP_TILE
#define LBM_STEP_TILE 128, 8, 4
#endif
using StepTile = TileShape<LBM_STEP_TILE>;

// Coordinates (hx, hy) in the (TY+2) x LW density tile of ring slot t.
template <class S>
__device__ __forceinline__ void ring_slot(int t, int& hx, int& hy) {
  if (t < S::LW) {
    hx = t, hy = 0;
  } else if (t < 2 * S::LW) {
    hx = t - S::LW, hy = S::TY + 1;
  } else if (t < 2 * S::LW + S::TY) {
    hx = 0, hy = t - 2 * S::LW + 1;
  } else {
    hx = S::LW - 1, hy = t - 2 * S::LW - S::TY + 1;
  }
}

// Populations of one tile held in registers: NPT own nodes per thread plus,
// for the first NRING threads, one ring node.
template <class S>
struct TileRegs {
  float f[S::NPT][9];
  float fr[9];
};

// Issue the loads of the tile at (x0, y0); ring loads first.
template <class S>
__device__ __forceinline__ void issue_tile(const Planes& P, int nx, int ny, int x0, int y0, TileRegs<S>& R) {
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * S::TX + tx;
  if (tid < S::NRING) {
    int hx, hy;
    ring_slot<S>(tid, hx, hy);
    pull9b(P, node_addr(wrap(x0 + hx - 1, nx), wrap(y0 + hy - 1, ny), nx, ny), R.fr);
  }
  const int xw = wrap(x0 + tx, nx);
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) pull9b(P, node_addr(xw, wrap(y0 + ty + k * S::WY, ny), nx, ny), R.f[k]);
}

// Densities of the tile and its ring into srho[(TY+2)][LW]; the exact
// (FP64) masses of the own nodes are kept for the collision.
template <class S>
__device__ __forceinline__ void stage_density(const TileRegs<S>& R, double (&mass)[S::NPT], float* srho) {
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * S::TX + tx;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    mass[k] = density_exact(R.f[k]);
    srho[(ty + k * S::WY + 1) * S::LW + tx + 1] = (float)mass[k];
  }
  if (tid < S::NRING) {
    int hx, hy;
    ring_slot<S>(tid, hx, hy);
    srho[hy * S::LW + hx] = density(R.fr);
  }
}

template <class S>
__device__ __forceinline__ void tile_gradient(const float* srho, int hx, int hy, float& gx, float& gy) {
  const float* r = srho + hy * S::LW + hx;
  stencil(r[1], r[S::LW], r[-1], r[-S::LW], r[S::LW + 1], r[S::LW - 1], r[-S::LW - 1], r[-S::LW + 1], gx, gy);
}

// Collide the own nodes of the tile at (x0, y0) and store f-bar at the node.
template <class S>
__device__ __forceinline__ void collide_tile(TileRegs<S>& R, const double (&mass)[S::NPT], const float* srho,
                                             const OutPlanes& Q, int nx, int ny, int x0, int y0,
                                             const Coef<float>& c) {
  const int x = x0 + threadIdx.x;
  if (x >= nx) return;
  const unsigned rb = 4u * (unsigned)nx;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    const int ly = threadIdx.y + k * S::WY, y = y0 + ly;
    if (y >= ny) break;
    float gx, gy;
    tile_gradient<S>(srho, threadIdx.x + 1, ly + 1, gx, gy);
    collide_node(R.f[k], mass[k], gx, gy, c);
    const unsigned o = rb * (unsigned)y + 4u * (unsigned)x;
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(R.f[k][i], reinterpret_cast<float*>(Q.p[i] + o));
  }
}

// Step kernel: one tile per workgroup, tiles ordered across the XCDs by
// xcd_tile so that neighbouring tiles (whose halo lines overlap) run on the
// same XCD and share its L2.
template <class S>
__global__ __launch_bounds__(S::NTHREADS) void step_f32(const float* __restrict__ src, float* __restrict__ dst,
                                                        int nx, int ny, int ntx, int ntiles, Coef<float> c) {
  __shared__ float srho[S::LDS];
  const size_t N = (size_t)nx * ny;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int x0 = (tile % ntx) * S::TX, y0 = (tile / ntx) * S::TY;
  TileRegs<S> R;
  double mass[S::NPT];
  issue_tile<S>(planes(src, N), nx, ny, x0, y0, R);
  stage_density<S>(R, mass, srho);
  __syncthreads();
  collide_tile<S>(R, mass, srho, out_planes(dst, N), nx, ny, x0, y0, c);
}

// Moments: rho and u of main Eq. 5 plus per-workgroup FP64 partial sums of
// mass and lattice momentum (reduced in a fixed order).
using MomTile = TileShape<64, 16, 4>;

__global__ __launch_bounds__(MomTile::NTHREADS) void moments_f32(const float* __restrict__ src,
                                                                 float* __restrict__ rho_out,
                                                                 float* __restrict__ ux_out,
                                                                 float* __restrict__ uy_out,
                                                                 double* __restrict__ partials, int nx, int ny,
                                                                 int ntx, Coef<float> c) {
  using S = MomTile;
  __shared__ float srho[S::LDS];
  __shared__ double sred[3][S::NTHREADS];
  const size_t N = (size_t)nx * ny;
  const int x0 = (blockIdx.x % ntx) * S::TX, y0 = (blockIdx.x / ntx) * S::TY;
  TileRegs<S> R;
  double mass[S::NPT];
  issue_tile<S>(planes(src, N), nx, ny, x0, y0, R);
  stage_density<S>(R, mass, srho);
  __syncthreads();
  auto& f = R.f;
  const int x = x0 + threadIdx.x;
  double sm = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
  for (int k = 0; k < S::NPT; ++k) {
    const int ly = threadIdx.y + k * S::WY, y = y0 + ly;
    if (x >= nx || y >= ny) continue;
    float m[9];
    forward_moments(f[k], m);
    float gx, gy;
    tile_gradient<S>(srho, threadIdx.x + 1, ly + 1, gx, gy);
    const NodeState<float> s = node_state(m[0], m[3], m[5], gx, gy, c);
    const size_t o = (size_t)y * nx + x;
    if (rho_out) rho_out[o] = m[0];
    if (ux_out) ux_out[o] = s.ux;
    if (uy_out) uy_out[o] = s.uy;
    sm += mass[k];
    sx += (double)m[3];
    sy += (double)m[5];
  }
  const int tid = threadIdx.y * S::TX + threadIdx.x;
  sred[0][tid] = sm;
  sred[1][tid] = sx;
  sred[2][tid] = sy;
  __syncthreads();
  for (int w = S::NTHREADS / 2; w > 0; w >>= 1) {
    if (tid < w) {
      sred[0][tid] += sred[0][tid + w];
      sred[1][tid] += sred[1][tid + w];
      sred[2][tid] += sred[2][tid + w];
    }
    __syncthreads();
  }
  if (tid < 3) partials[(size_t)blockIdx.x * 3 + tid] = sred[tid][0];
}

constexpr int RED = 256;
__global__ __launch_bounds__(RED) void finish_sums(const double* __restrict__ partials, int nblocks,
                                                   double* __restrict__ out) {
  __shared__ double s[3][RED];
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += RED)
    for (int k = 0; k < 3; ++k) a[k] += partials[(size_t)b * 3 + k];
  for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = RED / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = s[threadIdx.x][0];
}

// Initial state: node x computes f^eq(rho0, u0, eta(rho0)) and stores f_i at
// x - e_i, so that the first pull returns f^eq at x.  Raises *flag on a
// density outside (0, 4/b) or a non-finite input.
constexpr int BLK = 256;
__global__ __launch_bounds__(BLK) void init_f32(const float* __restrict__ rho0, const float* __restrict__ ux0,
                                                const float* __restrict__ uy0, float* __restrict__ dst, int nx,
                                                int ny, Coef<float> c, int* flag) {
  const size_t N = (size_t)nx * ny;
  const size_t o = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (o >= N) return;
  const int x = (int)(o % nx), y = (int)(o / nx);
  const float r = rho0[o], ux = ux0 ? ux0[o] : 0.0f, uy = uy0 ? uy0[o] : 0.0f;
  if (!(r > 0.0f && c.b4 * r < 1.0f) || !isfinite(ux) || !isfinite(uy)) atomicOr(flag, 1);
  float f[9];
  equilibrium_node(r, ux, uy, c, f);
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const size_t r0 = (size_t)y * nx, rm = (size_t)ym * nx, rp = (size_t)yp * nx;
  // population i stored at x - e_i
  dst[r0 + x] = f[0];
  dst[1 * N + r0 + xm] = f[1];
  dst[2 * N + rm + x] = f[2];
  dst[3 * N + r0 + xp] = f[3];
  dst[4 * N + rp + x] = f[4];
  dst[5 * N + rm + xm] = f[5];
  dst[6 * N + rm + xp] = f[6];
  dst[7 * N + rp + xp] = f[7];
  dst[8 * N + rp + xm] = f[8];
}

// Load a post-streaming state (un-stream it into the pull source layout).
__global__ __launch_bounds__(BLK) void set_state_f32(const float* __restrict__ fin, float* __restrict__ dst, int nx,
                                                     int ny) {
  const size_t N = (size_t)nx * ny;
  const size_t o = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (o >= N) return;
  const int x = (int)(o % nx), y = (int)(o / nx);
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const size_t r0 = (size_t)y * nx, rm = (size_t)ym * nx, rp = (size_t)yp * nx;
  dst[r0 + x] = fin[o];
  dst[1 * N + r0 + xm] = fin[1 * N + o];
  dst[2 * N + rm + x] = fin[2 * N + o];
  dst[3 * N + r0 + xp] = fin[3 * N + o];
  dst[4 * N + rp + x] = fin[4 * N + o];
  dst[5 * N + rm + xm] = fin[5 * N + o];
  dst[6 * N + rm + xp] = fin[6 * N + o];
  dst[7 * N + rp + xp] = fin[7 * N + o];
  dst[8 * N + rp + xm] = fin[8 * N + o];
}

__global__ __launch_bounds__(BLK) void get_state_f32(const float* __restrict__ src, float* __restrict__ fout, int nx,
                                                     int ny) {
  const size_t N = (size_t)nx * ny;
  const size_t o = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (o >= N) return;
  const int x = (int)(o % nx), y = (int)(o / nx);
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  float f[9];
  pull9(src, N, nx, x, xm, xp, y, ym, yp, f);
  for (int i = 0; i < 9; ++i) fout[i * N + o] = f[i];
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
  Coef<float> f;
  const double* src = reinterpret_cast<const double*>(&c);
  float* dstp = reinterpret_cast<float*>(&f);
  static_assert(sizeof(Coef<double>) == 2 * sizeof(Coef<float>), "Coef layout");
  for (size_t i = 0; i < sizeof(Coef<float>) / sizeof(float); ++i) dstp[i] = (float)src[i];
  return f;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_ctx {
  lbm_params p;
  lbm_derived d;
  Coef<float> c;
  void* buf[2];
  void* rho_ref;
  int cur;        // buffer holding the pull source of the next step
  bool ready;     // state initialised
  int64_t t;
  hipStream_t stream;
  int device;
  int nblocks;    // workgroups of the moments tile grid
  double* scratch;  // nblocks*3 partials, then 3 totals
  int* flag;
};

namespace {

template <class S>
int tiles_x(int nx) { return (nx + S::TX - 1) / S::TX; }
template <class S>
int tiles_total(int nx, int ny) { return tiles_x<S>(nx) * ((ny + S::TY - 1) / S::TY); }

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

size_t grid1(size_t n) { return (n + BLK - 1) / BLK; }

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
  return (size_t)9 * p->nx * p->ny * (p->storage == LBM_FP32 ? 4 : 2);
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
  if (p->storage != LBM_FP32) return fail(LBM_EINVAL, "this build supports LBM_FP32 storage only");
  if (!f_a || !f_b || f_a == f_b) return fail(LBM_EINVAL, "f_a and f_b must be two distinct device buffers");
  lbm_ctx* c = new (std::nothrow) lbm_ctx{};
  if (!c) return fail(LBM_EINVAL, "out of host memory");
  c->p = *p;
  c->d = d;
  c->c = make_coef(d, p->varpi, p->a, p->b);
  c->buf[0] = f_a;
  c->buf[1] = f_b;
  c->rho_ref = rho_ref;
  c->cur = 0;
  c->ready = false;
  c->t = 0;
  c->stream = (hipStream_t)stream;
  c->nblocks = tiles_total<MomTile>(p->nx, p->ny);
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipMalloc(&c->scratch, sizeof(double) * (3 * (size_t)c->nblocks + 3) + 64);
  if (e != hipSuccess) {
    delete c;
    return fail(LBM_EHIP, "lbm_create: %s", hipGetErrorString(e));
  }
  c->flag = reinterpret_cast<int*>(c->scratch + 3 * (size_t)c->nblocks + 3);
  *out = c;
  return LBM_OK;
}

int lbm_set_stream(lbm_ctx* ctx, void* stream) {
  if (int st = check_ctx(ctx, false)) return st;
  ctx->stream = (hipStream_t)stream;
  return LBM_OK;
}

int lbm_init(lbm_ctx* ctx, const float* rho0, const float* ux0, const float* uy0) {
  if (int st = check_ctx(ctx, false)) return st;
  if (!rho0) return fail(LBM_EINVAL, "rho0 is NULL");
  if (int st = set_device(ctx)) return st;
  const size_t N = (size_t)ctx->p.nx * ctx->p.ny;
  HIP_OK(hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream));
  float* dst = (float*)ctx->buf[0];
  init_f32<<<grid1(N), BLK, 0, ctx->stream>>>(rho0, ux0, uy0, dst, ctx->p.nx, ctx->p.ny, ctx->c, ctx->flag);
  HIP_OK(hipGetLastError());
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
  set_state_f32<<<grid1(N), BLK, 0, ctx->stream>>>(f, (float*)ctx->buf[0], ctx->p.nx, ctx->p.ny);
  HIP_OK(hipGetLastError());
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
  get_state_f32<<<grid1(N), BLK, 0, ctx->stream>>>((const float*)ctx->buf[ctx->cur], f, ctx->p.nx, ctx->p.ny);
  HIP_OK(hipGetLastError());
  return LBM_OK;
}

int lbm_step(lbm_ctx* ctx, int32_t n) {
  if (int st = check_ctx(ctx, true)) return st;
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  if (int st = set_device(ctx)) return st;
  using S = StepTile;
  const int ntx = tiles_x<S>(ctx->p.nx), ntiles = tiles_total<S>(ctx->p.nx, ctx->p.ny);
  const dim3 block(S::TX, S::WY);
  for (int32_t s = 0; s < n; ++s) {
    const float* src = (const float*)ctx->buf[ctx->cur];
    float* dst = (float*)ctx->buf[ctx->cur ^ 1];
    step_f32<S><<<ntiles, block, 0, ctx->stream>>>(src, dst, ctx->p.nx, ctx->p.ny, ntx, ntiles, ctx->c);
    ctx->cur ^= 1;
  }
  HIP_OK(hipGetLastError());
  ctx->t += n;
  return LBM_OK;
}

int lbm_moments(lbm_ctx* ctx, float* rho, float* ux, float* uy, double totals[3]) {
  if (int st = check_ctx(ctx, true)) return st;
  if (int st = set_device(ctx)) return st;
  using S = MomTile;
  moments_f32<<<tiles_total<S>(ctx->p.nx, ctx->p.ny), dim3(S::TX, S::WY), 0, ctx->stream>>>(
      (const float*)ctx->buf[ctx->cur], rho, ux, uy, ctx->scratch, ctx->p.nx, ctx->p.ny, tiles_x<S>(ctx->p.nx),
      ctx->c);
  HIP_OK(hipGetLastError());
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

int64_t lbm_time(const lbm_ctx* ctx) { return ctx ? ctx->t : -1; }

int lbm_get_derived(const lbm_ctx* ctx, lbm_derived* out) {
  if (int st = check_ctx(ctx, false)) return st;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = ctx->d;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  delete ctx;
}

}  // extern "C"
