// gfx950 kernels of the Cartesian SENSE normal operator, the FISTA step and the
// FP64 reductions.  Included once, by pfista_lib.hip.
//
// Data layout (all row-major, x fastest, complex64 interleaved):
//   image  x, y, w, z ...   [S][N][N]
//   coil maps               [S][C][N][N]
//   k-space data / t buffer [S][C][N][N]   (natural DFT order, DC at 0)
//   mask (2-D)              uint8 [S][N][N]; (phase-encode) uint8 [S][N] over ky
//
// Normal operator y = alpha A^H A x + beta w with A = M F S (F the unitary 2-D
// DFT) for a 2-D mask, in three passes over a per-coil buffer t:
//   k_row_fwd   t_c[y, :] = DFT_x(S_c[y, :] x[y, :])              (all rows, coils)
//   k_col       t_c[:, k] = IDFT_y(M[:, k] DFT_y t_c[:, k])       (in place)
//   k_row_inv   y[r, :]  = alpha sum_c conj(S_c[r, :]) IDFT_x t_c[r, :] + beta w
// For a phase-encode mask the x-transform pair cancels (F_x^H F_x = I) and one
// pass does everything: k_normal_1d.

#pragma once
#include "pfista_fft.hpp"

namespace pf {

// twiddle tables exp(-2 pi i m / N), m < N, for every supported N, FP64-computed
// on the host and rounded once to FP32
constexpr int kTwTotal = 64 + 128 + 160 + 192 + 256 + 320 + 384 + 512;
__device__ float2 g_tw[kTwTotal];

template <int N> struct TwOff;
template <> struct TwOff<64> { static constexpr int v = 0; };
template <> struct TwOff<128> { static constexpr int v = 64; };
template <> struct TwOff<160> { static constexpr int v = 192; };
template <> struct TwOff<192> { static constexpr int v = 352; };
template <> struct TwOff<256> { static constexpr int v = 544; };
template <> struct TwOff<320> { static constexpr int v = 800; };
template <> struct TwOff<384> { static constexpr int v = 1120; };
template <> struct TwOff<512> { static constexpr int v = 1504; };

// forward plan F and its mirror I (inverse); T = lanes per transform
template <int N> struct Plans;
template <> struct Plans<64> { using F = Plan<64, 8, 8, 8>; using I = Plan<64, 8, 8, 8>; };
template <> struct Plans<128> { using F = Plan<128, 8, 16, 8>; using I = Plan<128, 8, 8, 16>; };
template <> struct Plans<160> { using F = Plan<160, 16, 10, 16>; using I = Plan<160, 16, 16, 10>; };
template <> struct Plans<192> { using F = Plan<192, 16, 12, 16>; using I = Plan<192, 16, 16, 12>; };
template <> struct Plans<256> { using F = Plan<256, 16, 16, 16>; using I = Plan<256, 16, 16, 16>; };
template <> struct Plans<320> { using F = Plan<320, 16, 20, 4, 4>; using I = Plan<320, 16, 4, 4, 20>; };
template <> struct Plans<384> { using F = Plan<384, 16, 8, 8, 6>; using I = Plan<384, 16, 6, 8, 8>; };
template <> struct Plans<512> { using F = Plan<512, 16, 8, 8, 8>; using I = Plan<512, 16, 8, 8, 8>; };

template <int N> struct Geo {
  using F = typename Plans<N>::F;
  using I = typename Plans<N>::I;
  static constexpr int T = F::T;
  static_assert(I::T == T, "mirrored plans share T");
  static_assert(I::R_in == F::R_out && I::R_out == F::R_in, "plans must mirror");
  static constexpr int P = F::pmax() > I::pmax() ? F::pmax() : I::pmax();
  static constexpr int LDSN = LdsLen<N>::value;
  static constexpr int ROW_THREADS = 256;
  static constexpr int G = ROW_THREADS / T;   // transforms per row-pass workgroup
  static constexpr int COLS = 16;             // columns per column-pass workgroup
  static constexpr int COL_THREADS = COLS * T;
};

template <int N> __device__ __forceinline__ void load_twiddles(float2 *s_tw) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) s_tw[i] = g_tw[TwOff<N>::v + i];
}

// ---------------------------------------------------------------------------
// Pass 1: t_c[s, y, :] = DFT_x(S_c[s, y, :] * x[s, y, :]); task = (s, y, c), c fastest
template <int N>
__global__ __launch_bounds__(256) void k_row_fwd(const float2 *__restrict__ x,
                                                 const float2 *__restrict__ sens,
                                                 float2 *__restrict__ t, int C, int tasks) {
  using Gm = Geo<N>;
  using F = typename Gm::F;
  constexpr int T = Gm::T;
  __shared__ float2 s_tw[N];
  __shared__ float2 s_buf[Gm::G][Gm::LDSN];
  load_twiddles<N>(s_tw);
  const int g = threadIdx.x / T, j0 = threadIdx.x % T;
  const int task = blockIdx.x * Gm::G + g;
  const bool valid = task < tasks;
  const int c = valid ? task % C : 0;
  const int sy = valid ? task / C : 0;
  const int s = sy / N, yy = sy % N;
  const float2 *xr = x + (size_t)sy * N;
  const float2 *sr = sens + ((size_t)(s * C + c) * N + yy) * N;
  float2 v[Gm::P];
#pragma unroll
  for (int b = 0; b < F::NB_in; ++b) {
    const int j = j0 + b * T;
    const bool ok = valid && ((F::NB_in * T == F::B_in) || j < F::B_in);
#pragma unroll
    for (int r = 0; r < F::R_in; ++r) {
      const int i = j + r * F::B_in;
      v[b * F::R_in + r] = ok ? cmul(sr[i], xr[i]) : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  fft_run<F, -1>(v, s_buf[g], j0, s_tw);
  float2 *tr = t + ((size_t)(s * C + c) * N + yy) * N;
#pragma unroll
  for (int b = 0; b < F::NB_out; ++b) {
    const int j = j0 + b * T;
    if (valid && ((F::NB_out * T == F::B_out) || j < F::B_out)) {
#pragma unroll
      for (int r = 0; r < F::R_out; ++r) tr[j + r * F::B_out] = v[b * F::R_out + r];
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 2 (columns).  Block = 16 adjacent columns k of one (s, c); lane = col + 16 j0.
enum ColMode { COL_NORMAL = 0, COL_FWD_OUT = 1, COL_ADJ_IN = 2, COL_RESID = 3 };

template <int MASK1D> __device__ __forceinline__ bool sampled(const uint8_t *mask_s, int ky, int kx, int N) {
  return MASK1D ? mask_s[ky] != 0 : mask_s[(size_t)ky * N + kx] != 0;
}

template <int N, int MODE, int MASK1D>
__global__ __launch_bounds__(Geo<N>::COL_THREADS) void k_col(float2 *__restrict__ t,
                                                             const float2 *__restrict__ kin,
                                                             float2 *__restrict__ kout,
                                                             const uint8_t *__restrict__ mask, int C,
                                                             float a_scale, float b_scale,
                                                             double *__restrict__ partials) {
  using Gm = Geo<N>;
  using F = typename Gm::F;
  using I = typename Gm::I;
  constexpr int T = Gm::T;
  __shared__ float2 s_tw[N];
  __shared__ float2 s_buf[Gm::COLS][Gm::LDSN];
  __shared__ double s_red[Gm::COL_THREADS];
  load_twiddles<N>(s_tw);
  const int col = threadIdx.x % Gm::COLS, j0 = threadIdx.x / Gm::COLS;
  const int kx = blockIdx.x * Gm::COLS + col;
  const int sc = blockIdx.y;
  const int s = sc / C;
  const uint8_t *mask_s = MASK1D ? mask + (size_t)s * N : mask + (size_t)s * N * N;
  float2 *tc = t + (size_t)sc * N * N;
  float2 v[Gm::P];
  double acc = 0.0;

  if constexpr (MODE == COL_ADJ_IN) {
    // v = M b (masked k-space input) laid out as the inverse's inputs
    const float2 *kc = kin + (size_t)sc * N * N;
#pragma unroll
    for (int b = 0; b < I::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = (I::NB_in * T == I::B_in) || j < I::B_in;
#pragma unroll
      for (int r = 0; r < I::R_in; ++r) {
        const int ky = j + r * I::B_in;
        v[b * I::R_in + r] = (ok && sampled<MASK1D>(mask_s, ky, kx, N)) ? kc[(size_t)ky * N + kx]
                                                                         : make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int b = 0; b < F::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = (F::NB_in * T == F::B_in) || j < F::B_in;
#pragma unroll
      for (int r = 0; r < F::R_in; ++r) {
        const int yy = j + r * F::B_in;
        v[b * F::R_in + r] = ok ? tc[(size_t)yy * N + kx] : make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
    fft_run<F, -1>(v, s_buf[col], j0, s_tw);
    // registers now hold X[ky] for ky = j + r * F::B_out
#pragma unroll
    for (int b = 0; b < F::NB_out; ++b) {
      const int j = j0 + b * T;
      const bool ok = (F::NB_out * T == F::B_out) || j < F::B_out;
#pragma unroll
      for (int r = 0; r < F::R_out; ++r) {
        const int ky = j + r * F::B_out;
        float2 &e = v[b * F::R_out + r];
        const bool m = ok && sampled<MASK1D>(mask_s, ky, kx, N);
        if constexpr (MODE == COL_NORMAL) {
          if (!m) e = make_float2(0.f, 0.f);
        } else if constexpr (MODE == COL_FWD_OUT) {
          if (ok) kout[(size_t)sc * N * N + (size_t)ky * N + kx] = m ? cscale(e, a_scale) : make_float2(0.f, 0.f);
        } else if constexpr (MODE == COL_RESID) {
          if (m) {
            const float2 bb = kin[(size_t)sc * N * N + (size_t)ky * N + kx];
            const double rr = (double)e.x * a_scale - (double)bb.x * b_scale;
            const double ri = (double)e.y * a_scale - (double)bb.y * b_scale;
            acc += rr * rr + ri * ri;
          }
        }
      }
    }
  }

  if constexpr (MODE == COL_NORMAL || MODE == COL_ADJ_IN) {
    fft_run<I, +1>(v, s_buf[col], j0, s_tw);
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      if ((I::NB_out * T == I::B_out) || j < I::B_out) {
#pragma unroll
        for (int r = 0; r < I::R_out; ++r) tc[(size_t)(j + r * I::B_out) * N + kx] = v[b * I::R_out + r];
      }
    }
  }

  if constexpr (MODE == COL_RESID) {
    // deterministic block sum of the FP64 partials
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = Gm::COL_THREADS / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) s_red[threadIdx.x] += s_red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s_red[0];
  }
}

// ---------------------------------------------------------------------------
// Pass 3: y[s, r, :] = alpha sum_c conj(S_c[s, r, :]) IDFT_x(t_c[s, r, :]) + beta w.
// Block = RPW rows; transform group g handles row (g % RPW) and coils
// g / RPW, g / RPW + G / RPW, ...; groups are summed in a fixed order.
template <int N>
__global__ __launch_bounds__(256) void k_row_inv(const float2 *__restrict__ t,
                                                 const float2 *__restrict__ sens,
                                                 float2 *__restrict__ y, const float2 *w, float alpha,
                                                 float beta, int C, int rows, int rpw) {
  using Gm = Geo<N>;
  using I = typename Gm::I;
  constexpr int T = Gm::T;
  constexpr int G = Gm::G;
  __shared__ float2 s_tw[N];
  __shared__ float2 s_buf[G][Gm::LDSN];
  load_twiddles<N>(s_tw);
  const int g = threadIdx.x / T, j0 = threadIdx.x % T;
  const int ro = g % rpw, cg = g / rpw, cstep = G / rpw;
  const int row = blockIdx.x * rpw + ro;
  const bool rvalid = row < rows;
  const int s = rvalid ? row / N : 0, yy = rvalid ? row % N : 0;
  float2 acc[Gm::P];
#pragma unroll
  for (int i = 0; i < Gm::P; ++i) acc[i] = make_float2(0.f, 0.f);
  const int iters = (C + cstep - 1) / cstep;
  for (int it = 0; it < iters; ++it) {
    const int c = cg + it * cstep;
    const bool valid = rvalid && c < C;
    const size_t off = ((size_t)(s * C + (valid ? c : 0)) * N + yy) * N;
    const float2 *tr = t + off;
    float2 v[Gm::P];
#pragma unroll
    for (int b = 0; b < I::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && ((I::NB_in * T == I::B_in) || j < I::B_in);
#pragma unroll
      for (int r = 0; r < I::R_in; ++r) v[b * I::R_in + r] = ok ? tr[j + r * I::B_in] : make_float2(0.f, 0.f);
    }
    fft_run<I, +1>(v, s_buf[g], j0, s_tw);
    const float2 *sr = sens + off;
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && ((I::NB_out * T == I::B_out) || j < I::B_out);
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) {
        if (ok) acc[b * I::R_out + r] = cadd(acc[b * I::R_out + r], cmulc(v[b * I::R_out + r], sr[j + r * I::B_out]));
      }
    }
    __syncthreads();
  }
  // partial sums per group -> LDS (natural order), then fixed-order sum over coil groups
  float2 *red = &s_buf[0][0];
#pragma unroll
  for (int b = 0; b < I::NB_out; ++b) {
    const int j = j0 + b * T;
    if ((I::NB_out * T == I::B_out) || j < I::B_out) {
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) red[g * N + j + r * I::B_out] = acc[b * I::R_out + r];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rpw * N; e += blockDim.x) {
    const int r_o = e / N, i = e % N;
    const int rr = blockIdx.x * rpw + r_o;
    if (rr >= rows) continue;
    float2 sum = red[r_o * N + i];
    for (int q = 1; q < cstep; ++q) sum = cadd(sum, red[(q * rpw + r_o) * N + i]);
    float2 out = cscale(sum, alpha);
    const size_t o = (size_t)rr * N + i;
    if (w) out = cadd(out, cscale(w[o], beta));
    y[o] = out;
  }
}

// ---------------------------------------------------------------------------
// One-pass normal operator for a phase-encode mask (sampled rows ky, all kx):
// F^H M F = (F_y^H M_y F_y) (x) I, so each column only needs a y transform pair.
// Block = 16 columns of one slice, all coils accumulated in registers.
template <int N>
__global__ __launch_bounds__(Geo<N>::COL_THREADS) void k_normal_1d(const float2 *__restrict__ x,
                                                                   const float2 *__restrict__ sens,
                                                                   const uint8_t *__restrict__ mask,
                                                                   float2 *__restrict__ y,
                                                                   const float2 *w, float alpha,
                                                                   float beta, int C) {
  using Gm = Geo<N>;
  using F = typename Gm::F;
  using I = typename Gm::I;
  constexpr int T = Gm::T;
  __shared__ float2 s_tw[N];
  __shared__ float2 s_buf[Gm::COLS][Gm::LDSN];
  load_twiddles<N>(s_tw);
  const int col = threadIdx.x % Gm::COLS, j0 = threadIdx.x / Gm::COLS;
  const int kx = blockIdx.x * Gm::COLS + col;
  const int s = blockIdx.y;
  const uint8_t *mask_s = mask + (size_t)s * N;
  const float2 *xs = x + (size_t)s * N * N;
  // F's input layout == I's output layout: positions yy = j + r * F::B_in
  float2 xv[Gm::P], acc[Gm::P];
#pragma unroll
  for (int b = 0; b < F::NB_in; ++b) {
    const int j = j0 + b * T;
    const bool ok = (F::NB_in * T == F::B_in) || j < F::B_in;
#pragma unroll
    for (int r = 0; r < F::R_in; ++r) {
      xv[b * F::R_in + r] = ok ? xs[(size_t)(j + r * F::B_in) * N + kx] : make_float2(0.f, 0.f);
      acc[b * F::R_in + r] = make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  for (int c = 0; c < C; ++c) {
    const float2 *sc = sens + (size_t)(s * C + c) * N * N;
    float2 v[Gm::P];
#pragma unroll
    for (int b = 0; b < F::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = (F::NB_in * T == F::B_in) || j < F::B_in;
#pragma unroll
      for (int r = 0; r < F::R_in; ++r)
        v[b * F::R_in + r] = ok ? cmul(sc[(size_t)(j + r * F::B_in) * N + kx], xv[b * F::R_in + r])
                                : make_float2(0.f, 0.f);
    }
    fft_run<F, -1>(v, s_buf[col], j0, s_tw);
#pragma unroll
    for (int b = 0; b < F::NB_out; ++b) {
      const int j = j0 + b * T;
#pragma unroll
      for (int r = 0; r < F::R_out; ++r) {
        const int ky = j + r * F::B_out;
        if (!(((F::NB_out * T == F::B_out) || j < F::B_out) && mask_s[ky] != 0))
          v[b * F::R_out + r] = make_float2(0.f, 0.f);
      }
    }
    fft_run<I, +1>(v, s_buf[col], j0, s_tw);
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      const bool ok = (I::NB_out * T == I::B_out) || j < I::B_out;
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) {
        if (ok) {
          const float2 sv = sc[(size_t)(j + r * I::B_out) * N + kx];
          acc[b * I::R_out + r] = cadd(acc[b * I::R_out + r], cmulc(v[b * I::R_out + r], sv));
        }
      }
    }
    __syncthreads();
  }
  float2 *ys = y + (size_t)s * N * N;
  const float2 *ws = w ? w + (size_t)s * N * N : nullptr;
#pragma unroll
  for (int b = 0; b < I::NB_out; ++b) {
    const int j = j0 + b * T;
    if ((I::NB_out * T == I::B_out) || j < I::B_out) {
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) {
        const size_t o = (size_t)(j + r * I::B_out) * N + kx;
        float2 out = cscale(acc[b * I::R_out + r], alpha);
        if (ws) out = cadd(out, cscale(ws[o], beta));
        ys[o] = out;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fused FISTA step: v = z - pg_scale * pg; x_new = Psi^H soft(Psi v, lam) with an
// orthonormal L-level Haar Psi; z_new = x_new + beta (x_new - x_old); FP64
// partial sums of ||Psi x_new||_1, ||x_new - x_old||^2, ||x_new||^2.
// Block = one wave = a 16 x 16 pixel region; lane (tx, ty) owns a 2 x 2 block.
// Level 1 is in registers; level l >= 2 combines the 2 x 2 lane neighbourhood of
// stride 2^(l-2) by lane shuffles (every lane of a group computes the same
// coefficients, so the inverse is again local).
__device__ __forceinline__ float2 soft_thr(float2 w, float lam, double &l1) {
  const float m = sqrtf(w.x * w.x + w.y * w.y);
  if (m > lam) {
    const float sc = 1.0f - lam / m;
    l1 += (double)m - (double)lam;
    return make_float2(w.x * sc, w.y * sc);
  }
  return make_float2(0.f, 0.f);
}

__device__ __forceinline__ float2 shfl_xor2(float2 v, int m) {
  return make_float2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

struct Quad { float2 ll, dx, dy, dd; };
__device__ __forceinline__ Quad haar4(float2 a, float2 b, float2 c, float2 d) {
  // (LL, x-detail, y-detail, diagonal) of the 2 x 2 block [[a, b], [c, d]]
  const float2 ab = cadd(a, b), amb = csub(a, b), cd = cadd(c, d), cmd = csub(c, d);
  Quad q;
  q.ll = cscale(cadd(ab, cd), 0.5f);
  q.dx = cscale(cadd(amb, cmd), 0.5f);
  q.dy = cscale(csub(ab, cd), 0.5f);
  q.dd = cscale(csub(amb, cmd), 0.5f);
  return q;
}
__device__ __forceinline__ void ihaar4(const Quad &q, float2 &a, float2 &b, float2 &c, float2 &d) {
  const float2 s1 = cadd(q.ll, q.dy), d1 = csub(q.ll, q.dy);  // ll +- dy
  const float2 s2 = cadd(q.dx, q.dd), d2 = csub(q.dx, q.dd);  // dx +- dd
  a = cscale(cadd(s1, s2), 0.5f);   // ll + dx + dy + dd
  b = cscale(csub(s1, s2), 0.5f);   // ll - dx + dy - dd
  c = cscale(cadd(d1, d2), 0.5f);   // ll + dx - dy - dd
  d = cscale(csub(d1, d2), 0.5f);   // ll - dx - dy + dd
}

template <int LEVELS>
__global__ __launch_bounds__(64) void k_step(const float2 *__restrict__ z, const float2 *__restrict__ pg,
                                             const float2 *x_old, float2 *x_new, float2 *z_new,
                                             float pg_scale, float lam, float beta_arg,
                                             const int *__restrict__ k_dev, int N,
                                             double *__restrict__ partials) {
  const int lane = threadIdx.x, tx = lane & 7, ty = lane >> 3;
  const int s = blockIdx.z;
  const int px = blockIdx.x * 16 + 2 * tx, py = blockIdx.y * 16 + 2 * ty;
  const size_t o0 = (size_t)s * N * N + (size_t)py * N + px, o1 = o0 + N;
  float beta = beta_arg;
  if (k_dev) {
    const double k = (double)(*k_dev);
    beta = (float)(k / (k + 3.0));
  }
  const float4 z0 = *reinterpret_cast<const float4 *>(z + o0), z1 = *reinterpret_cast<const float4 *>(z + o1);
  const float4 g0 = *reinterpret_cast<const float4 *>(pg + o0), g1 = *reinterpret_cast<const float4 *>(pg + o1);
  const float4 q0 = *reinterpret_cast<const float4 *>(x_old + o0), q1 = *reinterpret_cast<const float4 *>(x_old + o1);
  const float2 a = make_float2(z0.x - pg_scale * g0.x, z0.y - pg_scale * g0.y);
  const float2 b = make_float2(z0.z - pg_scale * g0.z, z0.w - pg_scale * g0.w);
  const float2 c = make_float2(z1.x - pg_scale * g1.x, z1.y - pg_scale * g1.y);
  const float2 d = make_float2(z1.z - pg_scale * g1.z, z1.w - pg_scale * g1.w);
  double l1 = 0.0;
  Quad lev[LEVELS];
  Quad q = haar4(a, b, c, d);
  q.dx = soft_thr(q.dx, lam, l1);
  q.dy = soft_thr(q.dy, lam, l1);
  q.dd = soft_thr(q.dd, lam, l1);
  if (LEVELS == 1) q.ll = soft_thr(q.ll, lam, l1);
  lev[0] = q;
  float2 ll = q.ll;
#pragma unroll
  for (int l = 2; l <= LEVELS; ++l) {
    const int st = 1 << (l - 2);
    const int bx = (tx >> (l - 2)) & 1, by = (ty >> (l - 2)) & 1;
    const float2 ox = shfl_xor2(ll, st), oy = shfl_xor2(ll, 8 * st), od = shfl_xor2(ll, 9 * st);
    float2 A, B, Cc, D;
    if (!bx && !by) { A = ll; B = ox; Cc = oy; D = od; }
    else if (bx && !by) { A = ox; B = ll; Cc = od; D = oy; }
    else if (!bx && by) { A = oy; B = od; Cc = ll; D = ox; }
    else { A = od; B = oy; Cc = ox; D = ll; }
    Quad r = haar4(A, B, Cc, D);
    double l1g = 0.0;   // counted once per lane group
    r.dx = soft_thr(r.dx, lam, l1g);
    r.dy = soft_thr(r.dy, lam, l1g);
    r.dd = soft_thr(r.dd, lam, l1g);
    if (l == LEVELS) r.ll = soft_thr(r.ll, lam, l1g);
    if (!(tx & (2 * st - 1)) && !(ty & (2 * st - 1))) l1 += l1g;
    lev[l - 1] = r;
    ll = r.ll;
  }
#pragma unroll
  for (int l = LEVELS; l >= 2; --l) {
    Quad r = lev[l - 1];
    r.ll = ll;
    float2 A, B, Cc, D;
    ihaar4(r, A, B, Cc, D);
    const int bx = (tx >> (l - 2)) & 1, by = (ty >> (l - 2)) & 1;
    ll = (!bx && !by) ? A : (bx && !by) ? B : (!bx && by) ? Cc : D;
  }
  Quad r1 = lev[0];
  r1.ll = ll;
  float2 na, nb, nc, nd;
  ihaar4(r1, na, nb, nc, nd);
  const float2 oa = make_float2(q0.x, q0.y), ob = make_float2(q0.z, q0.w);
  const float2 oc = make_float2(q1.x, q1.y), od = make_float2(q1.z, q1.w);
  double dx2 = 0.0, xn2 = 0.0;
  auto acc = [&](float2 n, float2 o) {
    const double ex = (double)n.x - (double)o.x, ey = (double)n.y - (double)o.y;
    dx2 += ex * ex + ey * ey;
    xn2 += (double)n.x * n.x + (double)n.y * n.y;
  };
  acc(na, oa); acc(nb, ob); acc(nc, oc); acc(nd, od);
  auto mom = [&](float2 n, float2 o) {
    return make_float2(n.x + beta * (n.x - o.x), n.y + beta * (n.y - o.y));
  };
  const float2 za = mom(na, oa), zb = mom(nb, ob), zc = mom(nc, oc), zd = mom(nd, od);
  *reinterpret_cast<float4 *>(x_new + o0) = make_float4(na.x, na.y, nb.x, nb.y);
  *reinterpret_cast<float4 *>(x_new + o1) = make_float4(nc.x, nc.y, nd.x, nd.y);
  *reinterpret_cast<float4 *>(z_new + o0) = make_float4(za.x, za.y, zb.x, zb.y);
  *reinterpret_cast<float4 *>(z_new + o1) = make_float4(zc.x, zc.y, zd.x, zd.y);
  l1 = wave_sum(l1);
  dx2 = wave_sum(dx2);
  xn2 = wave_sum(xn2);
  if (lane == 0) {
    const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partials[3 * blk + 0] = l1;
    partials[3 * blk + 1] = dx2;
    partials[3 * blk + 2] = xn2;
  }
}

// ---------------------------------------------------------------------------
// Small helpers
// Sum `width`-strided FP64 partials in a fixed order into out[0..width).
// If hist != nullptr, also stores them at hist[(*k_dev) * width + ...] and
// advances the device iteration counter (the solver's step bookkeeping).
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partials, int count, int width,
                                                double *__restrict__ out, double *hist, int *k_dev,
                                                int hist_cap) {
  __shared__ double s[256];
  for (int c = 0; c < width; ++c) {
    double a = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) a += partials[(size_t)i * width + c];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      out[c] = s[0];
      if (hist && k_dev) {
        const int k = *k_dev;
        if (k < hist_cap) hist[(size_t)k * width + c] = s[0];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && k_dev) *k_dev = *k_dev + 1;
}

// FP64 partial sums of |v|^2 (grid-stride), one value per block
__global__ __launch_bounds__(256) void k_norm2(const float2 *__restrict__ v, size_t n,
                                               double *__restrict__ partials) {
  __shared__ double s[256];
  double a = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float2 e = v[i];
    a += (double)e.x * e.x + (double)e.y * e.y;
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_fill(float2 *__restrict__ v, size_t n, float2 val) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) v[i] = val;
}

// out = a * u  (may alias)
__global__ __launch_bounds__(256) void k_scale(const float2 *u, float2 *out, size_t n, float a) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    out[i] = cscale(u[i], a);
}

// v <- v / ||v|| using the FP64 norm held in norm2[0] (power iteration)
__global__ __launch_bounds__(256) void k_normalise(float2 *v, size_t n, const double *norm2) {
  const double nr = sqrt(norm2[0]);
  const float inv = nr > 0.0 ? (float)(1.0 / nr) : 0.0f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    v[i] = cscale(v[i], inv);
}

// Counter-based start vector for power iteration: SplitMix64 of (seed, index)
// mapped to [-1, 1) on both parts.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ __launch_bounds__(256) void k_random(float2 *v, size_t n, unsigned long long seed) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const unsigned long long h = splitmix64(seed * 0x100000001B3ull + 2 * i);
    const unsigned long long k = splitmix64(seed * 0x100000001B3ull + 2 * i + 1);
    v[i] = make_float2((float)((double)(h >> 11) * (1.0 / 4503599627370496.0) - 1.0),
                       (float)((double)(k >> 11) * (1.0 / 4503599627370496.0) - 1.0));
  }
}

}  // namespace pf
