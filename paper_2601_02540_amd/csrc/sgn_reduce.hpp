// sgn_reduce.hpp -- M-weighted totals (mass, energy, semi-discrete rates), the
// CFL speed maximum and the auxiliary-variable initialization.
//
// Totals follow Theorems 1 and 2: mass = 1^T M h, energy = 1^T M E with
// E = h((u^2+v^2)/2 + w^2/6 + g/2 (h+2b) + lambda/6 (eta/h-1)^2), and the
// rates 1^T M h_t and <d_q E, q_t>_M.  They are accumulated in FP64 whatever the
// storage type, each thread with a TwoSum-compensated accumulator, then
// combined by a fixed wave64 shuffle tree and a fixed cross-wave order; the
// per-block partials are combined by one final block in block order.  The
// result is therefore deterministic for a given grid.
#pragma once

#include "sgn_common.hpp"

namespace sgn {

constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 1024;

// Optional epilogue of the step tile: two compensated sums over the tile's
// owned nodes, written as 4 doubles per tile (sum, error, sum, error).
enum : int {
  EPI_NONE = 0,
  EPI_RELAX = 1,   // M s(1) and M s'(1) of relaxation RK4 (relax_node_terms at gam = 1)
  EPI_TOTALS = 2,  // M h and M E of the new state (mass and energy)
};

// Energy density h (u^2 + v^2)/2 + h w^2/6 + g h (h + 2b)/2 + lam h (eta/h - 1)^2/6
// of one node (Theorem 2's E, whose M-weighted sum is the total energy).
__device__ __forceinline__ double energy_density(double h, double u, double v, double w, double eta, double b,
                                                 double g, double lam) {
  const double rm1 = eta * (1.0 / h) - 1.0;
  const double e = w * w * (1.0 / 6.0) + 0.5 * g * (h + 2.0 * b) + lam * (1.0 / 6.0) * rm1 * rm1;
  return h * (0.5 * (u * u + v * v) + e);
}

// Relaxation RK4: one node's s(gam) = (e(q + gam d) - e(q)) / gam of the energy
// density e and its derivative s'(gam), from the node's values x, increments d
// and bottom b.  Each part of e is written out as a polynomial in gam (rational
// for the lambda term), so the difference is never formed by subtraction.
__device__ __forceinline__ void relax_node_terms(const double (&x)[5], const double (&dx)[5], double bb, double g,
                                                 double lam, double gam, double& s, double& ds) {
  const double h = x[0], u = x[1], v = x[2], w = x[3], eta = x[4], b = bb;
  const double dh = dx[0], du = dx[1], dv = dx[2], dw = dx[3], deta = dx[4];
  const double H = h + gam * dh;
  const double lin_uv = 2.0 * u * du + 2.0 * v * dv, sq_uv = du * du + dv * dv;
  const double lin_w = 2.0 * w * dw, sq_w = dw * dw;
  const double A = eta - h, B = deta - dh;
  const double Nl = h * (2.0 * A * B + gam * B * B) - dh * A * A;
  const double s_kin = 0.5 * (dh * (u * u + v * v) + H * (lin_uv + gam * sq_uv));
  const double s_w = (1.0 / 6.0) * (dh * w * w + H * (lin_w + gam * sq_w));
  const double s_pot = 0.5 * g * dh * (2.0 * h + 2.0 * b + gam * dh);
  const double ihH2 = 1.0 / (h * H * H);  // one division for both lambda terms
  const double s_lam = (lam / 6.0) * (Nl * H) * ihH2;
  const double d_kin = 0.5 * (dh * (lin_uv + gam * sq_uv) + H * sq_uv);
  const double d_w = (1.0 / 6.0) * (dh * (lin_w + gam * sq_w) + H * sq_w);
  const double d_pot = 0.5 * g * dh * dh;
  const double d_lam = (lam / 6.0) * (h * B * B * H - Nl * dh) * ihH2;
  s = s_kin + s_w + s_pot + s_lam;
  ds = d_kin + d_w + d_pot + d_lam;
}

__device__ __forceinline__ void wave_merge(CSum& a) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double s2 = __shfl_xor(a.s, off, 64);
    const double c2 = __shfl_xor(a.c, off, 64);
    a.merge(s2, c2);
  }
}

// Reduces NQ compensated accumulators over the block; thread 0 gets the result.
template <int NQ>
__device__ __forceinline__ void block_merge(CSum (&a)[NQ]) {
  __shared__ double sh[RED_THREADS / 64][NQ][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) wave_merge(a[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      sh[wave][q][0] = a[q].s;
      sh[wave][q][1] = a[q].c;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      a[q].init();
      for (int wv = 0; wv < RED_THREADS / 64; ++wv) a[q].merge(sh[wv][q][0], sh[wv][q][1]);
    }
  }
}

// WHAT = 0: (mass, energy) of state q.  WHAT = 1: (mass rate, energy rate)
// from state q and its right-hand side dq.
template <typename T, int WHAT>
__global__ __launch_bounds__(RED_THREADS) void totals_partial(const GridConst gc, const T* __restrict__ q,
                                                              const T* __restrict__ bplane,
                                                              const T* __restrict__ dq,
                                                              double* __restrict__ partials) {
  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const double g = gc.g, lam = gc.lam;
  CSum a[2];
  a[0].init();
  a[1].init();
  for (int j = blockIdx.x; j < ny; j += gridDim.x) {
    const double wy = axis_weight(j, ny, gc.bc_y, gc.dy);
    for (int i = threadIdx.x; i < nx; i += RED_THREADS) {
      const double M = axis_weight(i, nx, gc.bc_x, gc.dx) * wy;
      const size_t o = (size_t)j * nx + i;
      const double h = (double)q[o], u = (double)q[N + o], v = (double)q[2 * N + o];
      const double w = (double)q[3 * N + o], eta = (double)q[4 * N + o], b = (double)bplane[o];
      if (WHAT == 0) {
        a[0].add(M * h);
        a[1].add(M * energy_density(h, u, v, w, eta, b, g, lam));
      } else {
        const double r = eta * (1.0 / h);
        const double dEh = 0.5 * u * u + 0.5 * v * v + w * w * (1.0 / 6.0) + g * h + g * b +
                           lam * (1.0 / 6.0) * (1.0 - r * r);
        const double ht = (double)dq[o];
        const double rate = dEh * ht + h * u * (double)dq[N + o] + h * v * (double)dq[2 * N + o] +
                            h * w * (1.0 / 3.0) * (double)dq[3 * N + o] -
                            lam * (1.0 / 3.0) * (1.0 - r) * (double)dq[4 * N + o];
        a[0].add(M * ht);
        a[1].add(M * rate);
      }
    }
  }
  block_merge<2>(a);
  if (threadIdx.x == 0) {
    partials[4 * blockIdx.x + 0] = a[0].s;
    partials[4 * blockIdx.x + 1] = a[0].c;
    partials[4 * blockIdx.x + 2] = a[1].s;
    partials[4 * blockIdx.x + 3] = a[1].c;
  }
}

// Per-tile partials (4 doubles each: two compensated sums) of the step kernel's
// epilogue, reduced in two deterministic levels.  Level 1: block b merges
// partials [b per, min((b + 1) per, n)), thread t those at b per + t + 256 m.
static __global__ __launch_bounds__(RED_THREADS) void partials_merge(const double* __restrict__ in, int n, int per,
                                                              double* __restrict__ out) {
  CSum a[2];
  a[0].init();
  a[1].init();
  const int lo = blockIdx.x * per;
  const int hi = lo + per < n ? lo + per : n;
  for (int p = lo + threadIdx.x; p < hi; p += RED_THREADS) {
    a[0].merge(in[4 * p + 0], in[4 * p + 1]);
    a[1].merge(in[4 * p + 2], in[4 * p + 3]);
  }
  block_merge<2>(a);
  if (threadIdx.x == 0) {
    out[4 * blockIdx.x + 0] = a[0].s;
    out[4 * blockIdx.x + 1] = a[0].c;
    out[4 * blockIdx.x + 2] = a[1].s;
    out[4 * blockIdx.x + 3] = a[1].c;
  }
}

// Level 2 (one block): the two totals of the n level-1 partials go to
// series[2 k] and series[2 k + 1], k = *counter, and the counter advances.
static __global__ __launch_bounds__(RED_THREADS) void series_final(const double* __restrict__ in, int n,
                                                            double* __restrict__ series, int* __restrict__ counter) {
  CSum a[2];
  a[0].init();
  a[1].init();
  for (int p = threadIdx.x; p < n; p += RED_THREADS) {
    a[0].merge(in[4 * p + 0], in[4 * p + 1]);
    a[1].merge(in[4 * p + 2], in[4 * p + 3]);
  }
  block_merge<2>(a);
  if (threadIdx.x == 0) {
    const int k = *counter;
    series[2 * k] = a[0].s + a[0].c;
    series[2 * k + 1] = a[1].s + a[1].c;
    *counter = k + 1;
  }
}

// *counter = 0 (start of a recorded series).
static __global__ void counter_reset(int* __restrict__ counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// One block: combines nparts partials in block order; result[0..1] = totals.
static __global__ __launch_bounds__(RED_THREADS) void totals_final(const double* __restrict__ partials, int nparts,
                                                            double* __restrict__ result) {
  CSum a[2];
  a[0].init();
  a[1].init();
  for (int p = threadIdx.x; p < nparts; p += RED_THREADS) {
    a[0].merge(partials[4 * p + 0], partials[4 * p + 1]);
    a[1].merge(partials[4 * p + 2], partials[4 * p + 3]);
  }
  block_merge<2>(a);
  if (threadIdx.x == 0) {
    result[0] = a[0].s + a[0].c;
    result[1] = a[1].s + a[1].c;
  }
}

// Largest (|u|+c)/dx + (|v|+c)/dy with c^2 = g h + lambda eta^2 / (3 h^2).
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void speed_partial(const GridConst gc, const T* __restrict__ q,
                                                             double* __restrict__ partials) {
  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  double m = 0.0;
  for (int j = blockIdx.x; j < ny; j += gridDim.x) {
    for (int i = threadIdx.x; i < nx; i += RED_THREADS) {
      const size_t o = (size_t)j * nx + i;
      const double h = (double)q[o], u = (double)q[N + o], v = (double)q[2 * N + o], eta = (double)q[4 * N + o];
      const double c = sqrt(gc.g * h + gc.lam * eta * eta / (3.0 * h * h));
      const double sp = (fabs(u) + c) / gc.dx + (fabs(v) + c) / gc.dy;
      m = (sp > m || sp != sp) ? sp : m;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o2 = __shfl_xor(m, off, 64);
    m = (o2 > m || o2 != o2) ? o2 : m;
  }
  __shared__ double sh[RED_THREADS / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int wv = 1; wv < RED_THREADS / 64; ++wv) m = (sh[wv] > m || sh[wv] != sh[wv]) ? sh[wv] : m;
    partials[blockIdx.x] = m;
  }
}

static __global__ __launch_bounds__(RED_THREADS) void speed_final(const double* __restrict__ partials, int nparts,
                                                           double* __restrict__ result) {
  double m = 0.0;
  for (int p = threadIdx.x; p < nparts; p += RED_THREADS) m = (partials[p] > m || partials[p] != partials[p]) ? partials[p] : m;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o2 = __shfl_xor(m, off, 64);
    m = (o2 > m || o2 != o2) ? o2 : m;
  }
  __shared__ double sh[RED_THREADS / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int wv = 1; wv < RED_THREADS / 64; ++wv) m = (sh[wv] > m || sh[wv] != sh[wv]) ? sh[wv] : m;
    result[0] = m;
  }
}

// Auxiliary initialization (eq. (initialization)): eta = h,
// w = -h (D_x u + D_y v) + 3/2 (u D_x b + v D_y b), in place on q.
template <typename T>
__global__ __launch_bounds__(256) void init_aux_kernel(const GridConst gc, T* __restrict__ q,
                                                       const T* __restrict__ bplane) {
  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= nx || j >= ny) return;
  int im = i - 1, ip = i + 1, jm = j - 1, jp = j + 1;
  double sx = gc.inv2dx, sy = gc.inv2dy;
  if (gc.bc_x == BC_PERIODIC) {
    im = im < 0 ? nx - 1 : im;
    ip = ip >= nx ? 0 : ip;
  } else {
    if (i == 0) { im = 0; sx = gc.invdx; }
    if (i == nx - 1) { ip = nx - 1; sx = gc.invdx; }
  }
  if (gc.bc_y == BC_PERIODIC) {
    jm = jm < 0 ? ny - 1 : jm;
    jp = jp >= ny ? 0 : jp;
  } else {
    if (j == 0) { jm = 0; sy = gc.invdy; }
    if (j == ny - 1) { jp = ny - 1; sy = gc.invdy; }
  }
  const size_t o = (size_t)j * nx + i;
  const T* u = q + N;
  const T* v = q + 2 * N;
  const T h = q[o];
  const T Dxu = T(sx) * (u[(size_t)j * nx + ip] - u[(size_t)j * nx + im]);
  const T Dyv = T(sy) * (v[(size_t)jp * nx + i] - v[(size_t)jm * nx + i]);
  const T Dxb = T(sx) * (bplane[(size_t)j * nx + ip] - bplane[(size_t)j * nx + im]);
  const T Dyb = T(sy) * (bplane[(size_t)jp * nx + i] - bplane[(size_t)jm * nx + i]);
  q[3 * N + o] = -h * (Dxu + Dyv) + T(1.5) * (u[o] * Dxb + v[o] * Dyb);
  q[4 * N + o] = h;
}

}  // namespace sgn
