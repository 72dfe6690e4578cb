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
//
// Also here: the Toeplitz operator of a non-Cartesian trajectory (k_trow_fwd,
// k_tcol, k_trow_inv on 2N-point transforms, and the set-up kernels that build
// its kernel and the direct non-uniform DFTs); the fused FISTA step (k_step) and
// its pull-back for differentiation (k_prox_vjp, k_poly_combine_dot); FP64
// reductions, per slice for batches (k_reduce_seg).  Batch groups whose slices
// have different coil counts pass the cb / cs coil-image tables described below.

#pragma once
#include "pfista_fft.hpp"

namespace pf {

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

// Alternative radix schedules (variant 1) with twice the lanes per transform
// (fewer values per lane, more LDS hand-overs); a tuner may pick them per
// image side and coil count.
template <int N, int V> struct PlansV { using F = typename Plans<N>::F; using I = typename Plans<N>::I; };
template <> struct PlansV<64, 1> { using F = Plan<64, 16, 4, 4, 4>; using I = Plan<64, 16, 4, 4, 4>; };
template <> struct PlansV<128, 1> { using F = Plan<128, 16, 8, 4, 4>; using I = Plan<128, 16, 4, 4, 8>; };
template <> struct PlansV<160, 1> { using F = Plan<160, 16, 10, 4, 4>; using I = Plan<160, 16, 4, 4, 10>; };
template <> struct PlansV<192, 1> { using F = Plan<192, 16, 12, 4, 4>; using I = Plan<192, 16, 4, 4, 12>; };
template <> struct PlansV<256, 1> { using F = Plan<256, 32, 8, 8, 4>; using I = Plan<256, 32, 4, 8, 8>; };
template <> struct PlansV<320, 1> { using F = Plan<320, 32, 10, 4, 8>; using I = Plan<320, 32, 8, 4, 10>; };
template <> struct PlansV<384, 1> { using F = Plan<384, 32, 12, 8, 4>; using I = Plan<384, 32, 4, 8, 12>; };
template <> struct PlansV<512, 1> { using F = Plan<512, 32, 16, 4, 8>; using I = Plan<512, 32, 8, 4, 16>; };
constexpr int kVariants = 2;

// Plans of the one-pass phase-encode operator: fewer values per lane (more
// lanes per transform) keep its four per-lane arrays within two waves per SIMD.
template <int N> struct Plans1D { using F = typename Plans<N>::F; using I = typename Plans<N>::I; };
template <> struct Plans1D<384> { using F = Plan<384, 32, 12, 8, 4>; using I = Plan<384, 32, 4, 8, 12>; };
template <> struct Plans1D<320> { using F = Plan<320, 32, 10, 4, 8>; using I = Plan<320, 32, 8, 4, 10>; };
template <> struct Plans1D<512> { using F = Plan<512, 32, 16, 4, 8>; using I = Plan<512, 32, 8, 4, 16>; };

template <class F, class I, int WAVES = 4> struct PairGeo {
  static constexpr int N = F::N;
  static constexpr int T = F::T;
  static_assert(I::T == T && I::N == N, "mirrored plans share N and T");
  static_assert(I::R_in == F::R_out && I::R_out == F::R_in, "plans must mirror");
  static constexpr int P = F::pmax() > I::pmax() ? F::pmax() : I::pmax();
  static constexpr int P_IN = F::NB_in * F::R_in;     // == I::NB_out * I::R_out
  static constexpr int P_OUT = F::NB_out * F::R_out;  // == I::NB_in * I::R_in
  static_assert(P_IN == I::NB_out * I::R_out && P_OUT == I::NB_in * I::R_in, "layouts must match");
  static_assert(P_OUT <= 32, "mask bits must fit one word");
  static constexpr int LDSN = LdsLen<N>::value;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int G = THREADS / T;   // transforms per workgroup
  static constexpr int CPW = 64 / T;      // columns per wave in column kernels
  static constexpr int COLS = WAVES * CPW;  // columns per column-kernel workgroup
};
template <int N> struct TwBlock;
template <int N> struct TwBase;
template <int N, int V = 0> struct Geo : PairGeo<typename PlansV<N, V>::F, typename PlansV<N, V>::I> {
  using F = typename PlansV<N, V>::F;
  using I = typename PlansV<N, V>::I;
  // offsets of this geometry's forward / inverse twiddle tables in g_tw
  static constexpr int TWF = TwBase<N>::v + (V == 0 ? TwBlock<N>::f : TwBlock<N>::fa);
  static constexpr int TWI = TwBase<N>::v + (V == 0 ? TwBlock<N>::i : TwBlock<N>::ia);
};
// the phase-encode kernel's blocks span 16 columns (128 B of every row of a
// coil map) so that no cache line of the streamed coil maps is split between
// blocks
template <int N> struct Waves1D {
  static constexpr int v = 16 / (64 / Plans1D<N>::F::T);
};
template <int N> struct Geo1D : PairGeo<typename Plans1D<N>::F, typename Plans1D<N>::I, Waves1D<N>::v> {
  using F = typename Plans1D<N>::F;
  using I = typename Plans1D<N>::I;
};

// Twiddle tables of every plan (TwLayout order), FP64-computed on the host and
// rounded once to FP32; per image side N: [F][I][F 1-D][I 1-D][F alt][I alt].
template <int N> struct TwBlock {
  static constexpr int f = 0;
  static constexpr int i = f + TwLayout<typename Plans<N>::F>::size();
  static constexpr int f1 = i + TwLayout<typename Plans<N>::I>::size();
  static constexpr int i1 = f1 + TwLayout<typename Plans1D<N>::F>::size();
  static constexpr int fa = i1 + TwLayout<typename Plans1D<N>::I>::size();
  static constexpr int ia = fa + TwLayout<typename PlansV<N, 1>::F>::size();
  static constexpr int size = ia + TwLayout<typename PlansV<N, 1>::I>::size();
};
template <> struct TwBase<64> { static constexpr int v = 0; };
template <> struct TwBase<128> { static constexpr int v = TwBase<64>::v + TwBlock<64>::size; };
template <> struct TwBase<160> { static constexpr int v = TwBase<128>::v + TwBlock<128>::size; };
template <> struct TwBase<192> { static constexpr int v = TwBase<160>::v + TwBlock<160>::size; };
template <> struct TwBase<256> { static constexpr int v = TwBase<192>::v + TwBlock<192>::size; };
template <> struct TwBase<320> { static constexpr int v = TwBase<256>::v + TwBlock<256>::size; };
template <> struct TwBase<384> { static constexpr int v = TwBase<320>::v + TwBlock<320>::size; };
template <> struct TwBase<512> { static constexpr int v = TwBase<384>::v + TwBlock<384>::size; };
constexpr int kTwTotal = TwBase<512>::v + TwBlock<512>::size;
__device__ float2 g_tw[kTwTotal];

// copy `count` table entries starting at `off` into LDS (block-strided)
__device__ __forceinline__ void load_tw(float2 *dst, int off, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = g_tw[off + i];
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b to XCD b % 8), so
// consecutive blocks land on different L2s.  The row passes and the step number
// their blocks through xcd_block: block b takes work item (b % 8) * (nb / 8) +
// b / 8, which gives each XCD one contiguous eighth of the rows (of the step's
// tiles), the same eighth in every row pass and in the step; the rows a pass
// reads (coil maps, the step's output) are then the ones its XCD's L2 saw in the
// previous row-mapped kernel.  Any numbering is correct; this one is only faster.
// The inverse row passes of a batch group (the CB kernels) keep the plain numbering:
// there a row costs in proportion to its slice's coil count, and contiguous
// eighths would leave the XCD holding the many-coil slices running alone, while
// round-robin blocks spread every slice over all eight.  Passing nb = 1 selects
// the plain numbering.
__device__ __forceinline__ int xcd_block(int b, int nb) { return (nb % 8) ? b : (b % 8) * (nb / 8) + b / 8; }

// A twiddle table fetched into registers first and stored to LDS later: global
// loads issued in between stay in flight across the store (a load_tw right after
// them would wait for all of them).
template <int COUNT, int TH> struct TwRegs {
  static constexpr int K = (COUNT + TH - 1) / TH;
  float2 r[K];
  __device__ __forceinline__ void fetch(int off) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = (int)threadIdx.x + k * TH;
      if (i < COUNT) r[k] = g_tw[off + i];
    }
  }
  __device__ __forceinline__ void store(float2 *dst) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = (int)threadIdx.x + k * TH;
      if (i < COUNT) dst[i] = r[k];
    }
  }
};

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}


// Opaque copy of a lane index: keeps the compiler from hoisting every per-lane
// twiddle and LDS index of a transform out of a coil loop (which would pin them
// in registers for the whole loop); they are recomputed each iteration instead.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// register layouts: "in" = F's first stage = I's last stage; "out" = F's last = I's first
template <class PL> __device__ __forceinline__ bool lay_in_ok(int j) {
  return (PL::NB_in * PL::T == PL::B_in) || j < PL::B_in;
}
template <class PL> __device__ __forceinline__ bool lay_out_ok(int j) {
  return (PL::NB_out * PL::T == PL::B_out) || j < PL::B_out;
}

// ---------------------------------------------------------------------------
// Coil images: image ci of the coil-major buffers (coil maps, t, k-space) is
// coil ci - cb[s] of slice s = cs[ci].  cb == nullptr means every slice has C
// coils (ci = s * C + c); otherwise slice s owns images cb[s] .. cb[s+1]-1.

// Pass 1: t_c[s, y, :] = DFT_x(S_c[s, y, :] * x[s, y, :]); task = (s, y, c), c
// fastest, so the transform groups of a block share rows of x.  With per-slice
// coil counts slice s owns tasks cb[s]*N .. cb[s+1]*N - 1.
// A transform group is T consecutive lanes of one wave (wave-level hand-over).
// CB: the launch carries the per-slice image table cb (a batch group); the row
// kernels are also compiled without it, for launches whose slices share one
// coil count (cb = nullptr), so that those carry no table code.
template <int N, int V = 0, bool CB = false>
__global__ __launch_bounds__(256) void k_row_fwd(const float2 *__restrict__ x,
                                                 const float2 *__restrict__ sens,
                                                 float2 *__restrict__ t, int C, int tasks,
                                                 int *k_inc, const int *__restrict__ cb, int slices) {
  using Gm = Geo<N, V>;
  using F = typename Gm::F;
  // the solver's iteration counter: advanced here, read by the step kernel of
  // the same iteration (stream order separates the two)
  if (k_inc && blockIdx.x == 0 && threadIdx.x == 0) *k_inc += 1;
  if constexpr (!CB) cb = nullptr;
  constexpr int T = Gm::T;
  __shared__ float2 s_tw[TwLayout<F>::size()];
  __shared__ float2 s_buf[Gm::G][Gm::LDSN];
  const int g = threadIdx.x / T, j0 = threadIdx.x % T;
  const int task = xcd_block(blockIdx.x, gridDim.x) * Gm::G + g;
  const bool valid = task < tasks;
  int s, yy, cim;
  if (cb) {
    // the per-slice image table goes to LDS in one round trip (for up to
    // kRowCb - 1 slices), so the binary search below does not chain global loads
    constexpr int kRowCb = 257;
    __shared__ int s_cb[kRowCb];
    const bool in_lds = slices < kRowCb;
    if (in_lds) {
      for (int i = threadIdx.x; i <= slices; i += Gm::THREADS) s_cb[i] = cb[i];
      __syncthreads();
    }
    const int *tab = in_lds ? s_cb : cb;
    const int tk = valid ? task : 0;
    int lo = 0, hi = slices - 1;   // the slice whose task range holds tk
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab[mid] * N <= tk) lo = mid;
      else hi = mid - 1;
    }
    s = lo;
    const int base = tab[s], cnum = tab[s + 1] - base;
    const int local = tk - base * N;
    yy = local / cnum;
    cim = base + local % cnum;
  } else {
    const int c = valid ? task % C : 0;
    const int sy = valid ? task / C : 0;
    s = sy / N;
    yy = sy % N;
    cim = s * C + c;
  }
  const float2 *xr = x + ((size_t)s * N + yy) * N;
  const float2 *sr = sens + ((size_t)cim * N + yy) * N;
  // twiddles first: their LDS store and the barrier need not wait for the rows
  TwRegs<TwLayout<F>::size(), Gm::THREADS> twf;
  twf.fetch(Gm::TWF);
  float2 v[Gm::P];
#pragma unroll
  for (int b = 0; b < F::NB_in; ++b) {
    const int j = j0 + b * T;
    const bool ok = valid && lay_in_ok<F>(j);
#pragma unroll
    for (int r = 0; r < F::R_in; ++r) {
      const int i = j + r * F::B_in;
      v[b * F::R_in + r] = ok ? cmul(sr[i], xr[i]) : make_float2(0.f, 0.f);
    }
  }
  twf.store(s_tw);
  __syncthreads();
  fft_run<F, -1>(v, s_buf[g], j0, s_tw);
  float2 *tr = t + ((size_t)cim * N + yy) * N;
#pragma unroll
  for (int b = 0; b < F::NB_out; ++b) {
    const int j = j0 + b * T;
    if (valid && lay_out_ok<F>(j)) {
#pragma unroll
      for (int r = 0; r < F::R_out; ++r) tr[j + r * F::B_out] = v[b * F::R_out + r];
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 2 (columns).  Block = COLS adjacent columns k of one (s, c); wave w owns
// columns w*CPW .. w*CPW+CPW-1, lane = column + CPW * j0 inside the wave.
enum ColMode { COL_NORMAL = 0, COL_FWD_OUT = 1, COL_ADJ_IN = 2, COL_RESID = 3 };

template <int MASK1D> __device__ __forceinline__ bool sampled(const uint8_t *mask_s, int ky, int kx, int N) {
  return MASK1D ? mask_s[ky] != 0 : mask_s[(size_t)ky * N + kx] != 0;
}

template <int N, int MODE, int MASK1D, int V = 0>
__global__ __launch_bounds__(256, 2) void k_col(float2 *__restrict__ t, const float2 *__restrict__ kin,
                                             float2 *__restrict__ kout, const uint8_t *__restrict__ mask,
                                             int C, float a_scale, float b_scale,
                                             double *__restrict__ partials, const int *__restrict__ cs) {
  using Gm = Geo<N, V>;
  static_assert(N % Gm::COLS == 0, "column workgroups must tile the image side");
  using F = typename Gm::F;
  using I = typename Gm::I;
  constexpr int T = Gm::T;
  __shared__ float2 s_twF[TwLayout<F>::size()];
  __shared__ float2 s_twI[TwLayout<I>::size()];
  __shared__ float2 s_buf[Gm::COLS * Gm::LDSN];
  __shared__ double s_red[Gm::THREADS / 64];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int ci = ln % Gm::CPW, col = wv * Gm::CPW + ci, j0 = ln / Gm::CPW;
  // this column's exchange buffer: the wave's columns interleaved element by element
  float2 *bufc = s_buf + wv * Gm::CPW * Gm::LDSN + ci;
  const int kx = blockIdx.x * Gm::COLS + col;
  const int sc = blockIdx.y;
  const int s = cs ? cs[sc] : sc / C;
  const uint8_t *mask_s = MASK1D ? mask + (size_t)s * N : mask + (size_t)s * N * N;
  float2 *tc = t + (size_t)sc * N * N;
  float2 v[Gm::P];
  double acc = 0.0;

  // sampling flags at the k-space positions this lane holds (F's output layout)
  unsigned mbits = 0;

  if constexpr (MODE == COL_ADJ_IN) {
    // the flags decide which k-space values are read at all
#pragma unroll
    for (int b = 0; b < F::NB_out; ++b) {
      const int j = j0 + b * T;
#pragma unroll
      for (int r = 0; r < F::R_out; ++r)
        if (lay_out_ok<F>(j) && sampled<MASK1D>(mask_s, j + r * F::B_out, kx, N)) mbits |= 1u << (b * F::R_out + r);
    }
    const float2 *kc = kin + (size_t)sc * N * N;
#pragma unroll
    for (int b = 0; b < I::NB_in; ++b) {
      const int j = j0 + b * T;
#pragma unroll
      for (int r = 0; r < I::R_in; ++r) {
        const int ky = j + r * I::B_in;
        v[b * I::R_in + r] = ((mbits >> (b * I::R_in + r)) & 1u) ? kc[(size_t)ky * N + kx] : make_float2(0.f, 0.f);
      }
    }
    load_tw(s_twI, Gm::TWI, TwLayout<I>::size());
    __syncthreads();
  } else {
    // issue order: twiddles, the column, the mask bytes; the flags are needed
    // only after the forward transform, which runs while they arrive
    TwRegs<TwLayout<F>::size(), Gm::THREADS> twf;
    TwRegs<MODE == COL_NORMAL ? TwLayout<I>::size() : 1, Gm::THREADS> twi;
    twf.fetch(Gm::TWF);
    if constexpr (MODE == COL_NORMAL) twi.fetch(Gm::TWI);
#pragma unroll
    for (int b = 0; b < F::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = lay_in_ok<F>(j);
#pragma unroll
      for (int r = 0; r < F::R_in; ++r) {
        const int yy = j + r * F::B_in;
        v[b * F::R_in + r] = ok ? tc[(size_t)yy * N + kx] : make_float2(0.f, 0.f);
      }
    }
    uint8_t mb[F::NB_out * F::R_out];
#pragma unroll
    for (int b = 0; b < F::NB_out; ++b) {
      const int j = j0 + b * T;
#pragma unroll
      for (int r = 0; r < F::R_out; ++r) {
        const int ky = j + r * F::B_out;
        mb[b * F::R_out + r] =
            lay_out_ok<F>(j) ? (MASK1D ? mask_s[ky] : mask_s[(size_t)ky * N + kx]) : (uint8_t)0;
      }
    }
    twf.store(s_twF);
    if constexpr (MODE == COL_NORMAL) twi.store(s_twI);
    __syncthreads();
    fft_run<F, -1, Gm::CPW>(v, bufc, j0, s_twF);
#pragma unroll
    for (int i = 0; i < F::NB_out * F::R_out; ++i)
      if (mb[i] != 0) mbits |= 1u << i;
#pragma unroll
    for (int b = 0; b < F::NB_out; ++b) {
      const int j = j0 + b * T;
      const bool ok = lay_out_ok<F>(j);
#pragma unroll
      for (int r = 0; r < F::R_out; ++r) {
        const int ky = j + r * F::B_out;
        float2 &e = v[b * F::R_out + r];
        const bool m = (mbits >> (b * F::R_out + r)) & 1u;
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

  if constexpr (MODE == COL_NORMAL) {
    fft_run<I, +1, Gm::CPW>(v, bufc, j0, s_twI);
    // Output through the waves' exchange regions (column c of the block at
    // region c / CPW, element y at offset y * CPW + c % CPW), then written as
    // whole row segments, two adjacent columns per thread: a wave's direct store
    // would cover 32 bytes of each of 16 lines, and the block's four waves would
    // fill every line in four partial writes.
    constexpr int TPR = Gm::COLS / 2, RPI = Gm::THREADS / TPR, NL = (N + RPI - 1) / RPI;
    const int sq = threadIdx.x % TPR, sr0 = threadIdx.x / TPR;
    const float2 *ssrc = s_buf + (2 * sq / Gm::CPW) * Gm::CPW * Gm::LDSN + (2 * sq) % Gm::CPW;
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      if (lay_out_ok<I>(j)) {
#pragma unroll
        for (int r = 0; r < I::R_out; ++r) bufc[(j + r * I::B_out) * Gm::CPW] = v[b * I::R_out + r];
      }
    }
    __syncthreads();
    float4 *dst = reinterpret_cast<float4 *>(tc + blockIdx.x * Gm::COLS) + sq;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int yy = sr0 + k * RPI;
      if (yy < N) dst[(size_t)yy * (N / 2)] = *reinterpret_cast<const float4 *>(ssrc + yy * Gm::CPW);
    }
  }
  if constexpr (MODE == COL_ADJ_IN) {
    fft_run<I, +1, Gm::CPW>(v, bufc, j0, s_twI);
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      if (lay_out_ok<I>(j)) {
#pragma unroll
        for (int r = 0; r < I::R_out; ++r) tc[(size_t)(j + r * I::B_out) * N + kx] = v[b * I::R_out + r];
      }
    }
  }

  if constexpr (MODE == COL_RESID) {
    // deterministic block sum of the FP64 partials: wave sums, then waves in order
    acc = wave_sum_d(acc);
    if (ln == 0) s_red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = s_red[0];
#pragma unroll
      for (int q = 1; q < Gm::THREADS / 64; ++q) sum += s_red[q];
      partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// The combine of a block of rpw rows gives thread e the outputs e, e + blockDim,
// ...; its first w value is read together with the rows (at N = 256 with one row
// per block it is the only one), so the combine does not wait for it.
template <int N>
__device__ __forceinline__ float2 first_w(const float2 *w, int rpw, int rows, int nb) {
  if (!w || (int)threadIdx.x >= rpw * N) return make_float2(0.f, 0.f);
  const int rr = xcd_block(blockIdx.x, nb) * rpw + (int)threadIdx.x / N;
  return rr < rows ? w[(size_t)rr * N + threadIdx.x % N] : make_float2(0.f, 0.f);
}

// Pass 3: y[s, r, :] = alpha sum_c conj(S_c[s, r, :]) IDFT_x(t_c[s, r, :]) + beta w.
// Block = rpw rows; transform group g handles row (g % rpw) and coils
// g / rpw, g / rpw + G / rpw, ...; the groups are summed in a fixed order.
template <int N, int V = 0, bool CB = false>
__global__ __launch_bounds__(256, 2) void k_row_inv(const float2 *__restrict__ t,
                                                 const float2 *__restrict__ sens,
                                                 float2 *__restrict__ y, const float2 *w, float alpha,
                                                 float beta, int C, int rows, int rpw,
                                                 const int *__restrict__ cb) {
  using Gm = Geo<N, V>;
  using I = typename Gm::I;
  constexpr int T = Gm::T;
  constexpr int G = Gm::G;
  __shared__ float2 s_tw[TwLayout<I>::size()];
  __shared__ float2 s_buf[G][Gm::LDSN];
  const int g = threadIdx.x / T, j0 = threadIdx.x % T;
  const int ro = g % rpw, cg = g / rpw, cstep = G / rpw;
  if constexpr (!CB) cb = nullptr;
  const int nb = CB ? 1 : (int)gridDim.x;
  const int row = xcd_block(blockIdx.x, nb) * rpw + ro;
  const bool rvalid = row < rows;
  const int s = rvalid ? row / N : 0, yy = rvalid ? row % N : 0;
  // this slice's coil images (every row of a block lies in one slice: rpw divides N)
  const int cbase = cb ? cb[s] : s * C;
  const int Cs = cb ? cb[s + 1] - cbase : C;
  float2 acc[Gm::P_IN];
#pragma unroll
  for (int i = 0; i < Gm::P_IN; ++i) acc[i] = make_float2(0.f, 0.f);
  // twiddles first: their LDS store then waits for them alone, not for the rows
  TwRegs<TwLayout<I>::size(), Gm::THREADS> twi;
  twi.fetch(Gm::TWI);
  float2 w0 = make_float2(0.f, 0.f);   // this thread's first w value of the combine
  const int iters = (Cs + cstep - 1) / cstep;
  for (int it = 0; it < iters; ++it) {
    const int c = cg + it * cstep;
    const bool valid = rvalid && c < Cs;
    const size_t off = ((size_t)(cbase + (valid ? c : 0)) * N + yy) * N;
    const float2 *tr = t + off;
    const float2 *sr = sens + off;
    float2 v[Gm::P], sv[Gm::P_IN];
#pragma unroll
    for (int b = 0; b < I::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && lay_in_ok<I>(j);
#pragma unroll
      for (int r = 0; r < I::R_in; ++r) v[b * I::R_in + r] = ok ? tr[j + r * I::B_in] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && lay_out_ok<I>(j);
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) sv[b * I::R_out + r] = ok ? sr[j + r * I::B_out] : make_float2(0.f, 0.f);
    }
    if (it == 0) {
      w0 = first_w<N>(w, rpw, rows, nb);
      twi.store(s_tw);
      __syncthreads();
    }
    fft_run<I, +1>(v, s_buf[opaque(g)], opaque(j0), s_tw);
#pragma unroll
    for (int i = 0; i < Gm::P_IN; ++i) acc[i] = cadd(acc[i], cmulc(v[i], sv[i]));
  }
  __syncthreads();
  // partial sums per group -> LDS (natural order), then fixed-order sum over coil groups
  float2 *red = &s_buf[0][0];
#pragma unroll
  for (int b = 0; b < I::NB_out; ++b) {
    const int j = j0 + b * T;
    if (lay_out_ok<I>(j)) {
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) red[g * N + j + r * I::B_out] = acc[b * I::R_out + r];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rpw * N; e += blockDim.x) {
    const int r_o = e / N, i = e % N;
    const int rr = xcd_block(blockIdx.x, nb) * rpw + r_o;
    if (rr >= rows) continue;
    float2 sum = red[r_o * N + i];
    for (int q = 1; q < cstep; ++q) sum = cadd(sum, red[(q * rpw + r_o) * N + i]);
    float2 out = cscale(sum, alpha);
    const size_t o = (size_t)rr * N + i;
    if (w) out = cadd(out, cscale(e == (int)threadIdx.x ? w0 : w[o], beta));
    y[o] = out;
  }
}

// ---------------------------------------------------------------------------
// Pass 3 of one apply fused with pass 1 of the next (the Horner chain feeds each
// output straight back in): for every row r
//   y[s, r, :] = alpha sum_c conj(S_c) IDFT_x(t_c[s, r, :]) + beta w[s, r, :]
//   t_c[s, r, :] = DFT_x(S_c[s, r, :] y[s, r, :])            (in place)
// The row's coil maps are read once for both halves.
template <int N, int V = 0, bool CB = false>
__global__ __launch_bounds__(256, 2) void k_row_inv_fwd(float2 *__restrict__ t, const float2 *__restrict__ sens,
                                                        float2 *__restrict__ y, const float2 *w, float alpha,
                                                        float beta, int C, int rows, int rpw,
                                                        const int *__restrict__ cb) {
  using Gm = Geo<N, V>;
  using F = typename Gm::F;
  using I = typename Gm::I;
  constexpr int T = Gm::T;
  constexpr int G = Gm::G;
  static_assert(Gm::P_IN == F::NB_in * F::R_in, "layouts");
  __shared__ float2 s_twF[TwLayout<F>::size()];
  __shared__ float2 s_twI[TwLayout<I>::size()];
  __shared__ float2 s_buf[G][Gm::LDSN];
  const int g = threadIdx.x / T, j0 = threadIdx.x % T;
  const int ro = g % rpw, cg = g / rpw, cstep = G / rpw;
  if constexpr (!CB) cb = nullptr;
  const int nb = CB ? 1 : (int)gridDim.x;
  const int row = xcd_block(blockIdx.x, nb) * rpw + ro;
  const bool rvalid = row < rows;
  const int s = rvalid ? row / N : 0, yy = rvalid ? row % N : 0;
  const int cbase = cb ? cb[s] : s * C;
  const int Cs = cb ? cb[s + 1] - cbase : C;
  float2 acc[Gm::P_IN], sv[Gm::P_IN];
#pragma unroll
  for (int i = 0; i < Gm::P_IN; ++i) acc[i] = make_float2(0.f, 0.f);
  // twiddles first: their LDS store then waits for them alone, not for the rows
  TwRegs<TwLayout<I>::size(), Gm::THREADS> twi;
  TwRegs<TwLayout<F>::size(), Gm::THREADS> twf;
  twi.fetch(Gm::TWI);
  twf.fetch(Gm::TWF);
  float2 w0 = make_float2(0.f, 0.f);   // this thread's first w value of the combine
  const int iters = (Cs + cstep - 1) / cstep;
  for (int it = 0; it < iters; ++it) {
    const int c = cg + it * cstep;
    const bool valid = rvalid && c < Cs;
    const size_t off = ((size_t)(cbase + (valid ? c : 0)) * N + yy) * N;
    const float2 *tr = t + off;
    const float2 *sr = sens + off;
    float2 v[Gm::P];
#pragma unroll
    for (int b = 0; b < I::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && lay_in_ok<I>(j);
#pragma unroll
      for (int r = 0; r < I::R_in; ++r) v[b * I::R_in + r] = ok ? tr[j + r * I::B_in] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && lay_out_ok<I>(j);
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) sv[b * I::R_out + r] = ok ? sr[j + r * I::B_out] : make_float2(0.f, 0.f);
    }
    if (it == 0) {
      w0 = first_w<N>(w, rpw, rows, nb);
      twi.store(s_twI);
      twf.store(s_twF);
      __syncthreads();
    }
    fft_run<I, +1>(v, s_buf[opaque(g)], opaque(j0), s_twI);
#pragma unroll
    for (int i = 0; i < Gm::P_IN; ++i) acc[i] = cadd(acc[i], cmulc(v[i], sv[i]));
  }
  __syncthreads();
  float2 *red = &s_buf[0][0];
#pragma unroll
  for (int b = 0; b < I::NB_out; ++b) {
    const int j = j0 + b * T;
    if (lay_out_ok<I>(j)) {
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) red[g * N + j + r * I::B_out] = acc[b * I::R_out + r];
    }
  }
  __syncthreads();
  // combined rows: written out, and kept for the forward half in their own LDS
  // rows when they fit (then the forward exchanges, which reuse the partial-sum
  // area, need not wait for every group to have read them), else in the q = 0
  // slot of each row
  constexpr int KC = N <= 384 ? 2 * N : 1;
  __shared__ float2 s_comb[KC];
  const bool sep = rpw * N <= KC;
  float2 *comb = sep ? s_comb : red;
  for (int e = threadIdx.x; e < rpw * N; e += blockDim.x) {
    const int r_o = e / N, i = e % N;
    const int rr = xcd_block(blockIdx.x, nb) * rpw + r_o;
    float2 sum = red[r_o * N + i];
    for (int q = 1; q < cstep; ++q) sum = cadd(sum, red[(q * rpw + r_o) * N + i]);
    float2 out = cscale(sum, alpha);
    if (rr < rows) {
      const size_t o = (size_t)rr * N + i;
      if (w) out = cadd(out, cscale(e == (int)threadIdx.x ? w0 : w[o], beta));
      y[o] = out;
    }
    comb[r_o * N + i] = out;
  }
  __syncthreads();
  float2 yv[Gm::P_IN];
#pragma unroll
  for (int b = 0; b < F::NB_in; ++b) {
    const int j = j0 + b * T;
#pragma unroll
    for (int r = 0; r < F::R_in; ++r) yv[b * F::R_in + r] = lay_in_ok<F>(j) ? comb[ro * N + j + r * F::B_in] : make_float2(0.f, 0.f);
  }
  if (!sep) __syncthreads();
  for (int it = 0; it < iters; ++it) {
    const int c = cg + it * cstep;
    const bool valid = rvalid && c < Cs;
    const size_t off = ((size_t)(cbase + (valid ? c : 0)) * N + yy) * N;
    if (iters > 1) {
      const float2 *sr = sens + off;
#pragma unroll
      for (int b = 0; b < F::NB_in; ++b) {
        const int j = j0 + b * T;
        const bool ok = valid && lay_in_ok<F>(j);
#pragma unroll
        for (int r = 0; r < F::R_in; ++r) sv[b * F::R_in + r] = ok ? sr[j + r * F::B_in] : make_float2(0.f, 0.f);
      }
    }
    float2 v[Gm::P];
#pragma unroll
    for (int i = 0; i < Gm::P_IN; ++i) v[i] = cmul(sv[i], yv[i]);
    fft_run<F, -1>(v, s_buf[opaque(g)], opaque(j0), s_twF);
    float2 *tr = t + off;
#pragma unroll
    for (int b = 0; b < F::NB_out; ++b) {
      const int j = j0 + b * T;
      if (valid && lay_out_ok<F>(j)) {
#pragma unroll
        for (int r = 0; r < F::R_out; ++r) tr[j + r * F::B_out] = v[b * F::R_out + r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Toeplitz normal operator of a non-Cartesian trajectory: for every coil image
//   y += conj(S_c) crop_N(IDFT_M(K DFT_M(pad_M(S_c x)))),  M = 2N,
// with the real M x M kernel K of the trajectory, in three passes over a
// per-coil buffer t [S][C][N][M] (only the N image rows; rows N..M-1 of the
// padded image are zero and are never stored).
//   k_trow_fwd   t_c[y, :] = DFT_M(pad(S_c[y, :] x[y, :]))      (y < N)
//   k_tcol       t_c[:, k] = crop_N(IDFT_M(K[:, k] DFT_M(pad t_c[:, k])))
//   k_trow_inv   y[r, :]  = alpha sum_c conj(S_c[r, :]) crop_N(IDFT_M t_c[r, :]) + beta w
template <int M>
__global__ __launch_bounds__(256) void k_trow_fwd(const float2 *__restrict__ x, const float2 *__restrict__ sens,
                                                  float2 *__restrict__ t, int C, int tasks, int *k_inc) {
  using Gm = Geo<M>;
  using F = typename Gm::F;
  constexpr int N = M / 2;
  constexpr int T = Gm::T;
  if (k_inc && blockIdx.x == 0 && threadIdx.x == 0) *k_inc += 1;
  __shared__ float2 s_tw[TwLayout<F>::size()];
  __shared__ float2 s_buf[Gm::G][Gm::LDSN];
  const int g = threadIdx.x / T, j0 = threadIdx.x % T;
  const int task = blockIdx.x * Gm::G + g;
  const bool valid = task < tasks;
  const int c = valid ? task % C : 0;
  const int sy = valid ? task / C : 0;
  const int s = sy / N, yy = sy % N;
  const float2 *xr = x + (size_t)sy * N;
  const float2 *sr = sens + ((size_t)(s * C + c) * N + yy) * N;
  TwRegs<TwLayout<F>::size(), Gm::THREADS> twf;   // twiddles first (see TwRegs)
  twf.fetch(Gm::TWF);
  float2 v[Gm::P];
#pragma unroll
  for (int b = 0; b < F::NB_in; ++b) {
    const int j = j0 + b * T;
    const bool ok = valid && lay_in_ok<F>(j);
#pragma unroll
    for (int r = 0; r < F::R_in; ++r) {
      const int i = j + r * F::B_in;
      v[b * F::R_in + r] = (ok && i < N) ? cmul(sr[i], xr[i]) : make_float2(0.f, 0.f);
    }
  }
  twf.store(s_tw);
  __syncthreads();
  fft_run<F, -1>(v, s_buf[g], j0, s_tw);
  float2 *tr = t + ((size_t)(s * C + c) * N + yy) * M;
#pragma unroll
  for (int b = 0; b < F::NB_out; ++b) {
    const int j = j0 + b * T;
    if (valid && lay_out_ok<F>(j)) {
#pragma unroll
      for (int r = 0; r < F::R_out; ++r) tr[j + r * F::B_out] = v[b * F::R_out + r];
    }
  }
}

template <int M>
__global__ __launch_bounds__(256, 2) void k_tcol(float2 *__restrict__ t, const float *__restrict__ kern, int C) {
  using Gm = Geo<M>;
  using F = typename Gm::F;
  using I = typename Gm::I;
  constexpr int N = M / 2;
  constexpr int T = Gm::T;
  __shared__ float2 s_twF[TwLayout<F>::size()];
  __shared__ float2 s_twI[TwLayout<I>::size()];
  __shared__ float2 s_buf[Gm::COLS * Gm::LDSN];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int ci = ln % Gm::CPW, col = wv * Gm::CPW + ci, j0 = ln / Gm::CPW;
  float2 *bufc = s_buf + wv * Gm::CPW * Gm::LDSN + ci;
  const int kx = blockIdx.x * Gm::COLS + col;
  const int sc = blockIdx.y;
  const int s = sc / C;
  const float *ks = kern + (size_t)s * M * M;
  float2 *tc = t + (size_t)sc * N * M;
  float2 v[Gm::P];
#pragma unroll
  for (int b = 0; b < F::NB_in; ++b) {
    const int j = j0 + b * T;
    const bool ok = lay_in_ok<F>(j);
#pragma unroll
    for (int r = 0; r < F::R_in; ++r) {
      const int yy = j + r * F::B_in;
      v[b * F::R_in + r] = (ok && yy < N) ? tc[(size_t)yy * M + kx] : make_float2(0.f, 0.f);
    }
  }
  // (the kernel values are read after the forward transform: fetching them with
  // the column measured slower, 15.3 against 14.1 us at M = 512)
  load_tw(s_twF, Gm::TWF, TwLayout<F>::size());
  load_tw(s_twI, Gm::TWI, TwLayout<I>::size());
  __syncthreads();
  fft_run<F, -1, Gm::CPW>(v, bufc, j0, s_twF);
#pragma unroll
  for (int b = 0; b < F::NB_out; ++b) {
    const int j = j0 + b * T;
    const bool ok = lay_out_ok<F>(j);
#pragma unroll
    for (int r = 0; r < F::R_out; ++r) {
      const int ky = j + r * F::B_out;
      const float kv = ok ? ks[(size_t)ky * M + kx] : 0.f;
      v[b * F::R_out + r] = cscale(v[b * F::R_out + r], kv);
    }
  }
  fft_run<I, +1, Gm::CPW>(v, bufc, j0, s_twI);
#pragma unroll
  for (int b = 0; b < I::NB_out; ++b) {
    const int j = j0 + b * T;
    if (lay_out_ok<I>(j)) {
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) {
        const int yy = j + r * I::B_out;
        if (yy < N) tc[(size_t)yy * M + kx] = v[b * I::R_out + r];
      }
    }
  }
}

template <int M>
__global__ __launch_bounds__(256, 2) void k_trow_inv(const float2 *__restrict__ t, const float2 *__restrict__ sens,
                                                   float2 *__restrict__ y, const float2 *w, float alpha, float beta,
                                                   int C, int rows, int rpw) {
  using Gm = Geo<M>;
  using I = typename Gm::I;
  constexpr int N = M / 2;
  constexpr int T = Gm::T;
  constexpr int G = Gm::G;
  __shared__ float2 s_tw[TwLayout<I>::size()];
  __shared__ float2 s_buf[G][Gm::LDSN];
  const int g = threadIdx.x / T, j0 = threadIdx.x % T;
  const int ro = g % rpw, cg = g / rpw, cstep = G / rpw;
  const int row = blockIdx.x * rpw + ro;
  const bool rvalid = row < rows;
  const int s = rvalid ? row / N : 0, yy = rvalid ? row % N : 0;
  float2 acc[Gm::P_IN];
#pragma unroll
  for (int i = 0; i < Gm::P_IN; ++i) acc[i] = make_float2(0.f, 0.f);
  TwRegs<TwLayout<I>::size(), Gm::THREADS> twi;   // twiddles first (see TwRegs)
  twi.fetch(Gm::TWI);
  const int iters = (C + cstep - 1) / cstep;
  for (int it = 0; it < iters; ++it) {
    const int c = cg + it * cstep;
    const bool valid = rvalid && c < C;
    const size_t cimg = (size_t)(s * C + (valid ? c : 0)) * N + yy;
    const float2 *tr = t + cimg * M;
    const float2 *sr = sens + cimg * N;
    float2 v[Gm::P], sv[Gm::P_IN];
#pragma unroll
    for (int b = 0; b < I::NB_in; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && lay_in_ok<I>(j);
#pragma unroll
      for (int r = 0; r < I::R_in; ++r) v[b * I::R_in + r] = ok ? tr[j + r * I::B_in] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int b = 0; b < I::NB_out; ++b) {
      const int j = j0 + b * T;
      const bool ok = valid && lay_out_ok<I>(j);
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) {
        const int i = j + r * I::B_out;
        sv[b * I::R_out + r] = (ok && i < N) ? sr[i] : make_float2(0.f, 0.f);
      }
    }
    if (it == 0) {
      twi.store(s_tw);
      __syncthreads();
    }
    fft_run<I, +1>(v, s_buf[opaque(g)], opaque(j0), s_tw);
#pragma unroll
    for (int i = 0; i < Gm::P_IN; ++i) acc[i] = cadd(acc[i], cmulc(v[i], sv[i]));
  }
  __syncthreads();
  float2 *red = &s_buf[0][0];
#pragma unroll
  for (int b = 0; b < I::NB_out; ++b) {
    const int j = j0 + b * T;
    if (lay_out_ok<I>(j)) {
#pragma unroll
      for (int r = 0; r < I::R_out; ++r) {
        const int i = j + r * I::B_out;
        if (i < N) red[g * N + i] = acc[b * I::R_out + r];
      }
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

// Kernel of the Toeplitz operator from a trajectory (cycles per field of view,
// [S][J][2]) and optional weights [S][J]:
//   K[ky][kx] = (1/n^2) sum_j w_j D(kx_j/n - kx/2n) D(ky_j/n - ky/2n),
//   D(u) = sum_{m=-(n-1)}^{n-1} exp(2 pi i m u) = sin((2n-1) pi u) / sin(pi u),
// the DFT of the difference kernel h(m) = (1/n^2) sum_j w_j exp(2 pi i k_j.m/n)
// on the 2n grid.  FP64 throughout; one thread per (slice, ky, kx).
__device__ __forceinline__ double dirichlet(double u, int n) {
  const double r = u - rint(u);                  // D has period 1 in u
  const double sr = sin(M_PI * r);
  if (fabs(sr) < 1e-9) return (double)(2 * n - 1);   // D(0) = 2n - 1 (2n - 1 is odd)
  return sin((2 * n - 1) * M_PI * r) / sr;
}

__global__ __launch_bounds__(256) void k_toeplitz_kernel(const float *__restrict__ traj, const float *weights,
                                                         int J, int n, int slices, float *__restrict__ kern) {
  const int m = 2 * n;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)slices * m * m) return;
  const int s = (int)(idx / ((size_t)m * m));
  const int rem = (int)(idx % ((size_t)m * m));
  const int ky = rem / m, kx = rem % m;
  const float *ts = traj + (size_t)s * J * 2;
  const float *ws = weights ? weights + (size_t)s * J : nullptr;
  double acc = 0.0;
  for (int j = 0; j < J; ++j) {
    const double ax = (double)ts[2 * j] / n - (double)kx / m;
    const double ay = (double)ts[2 * j + 1] / n - (double)ky / m;
    const double wj = ws ? (double)ws[j] : 1.0;
    acc += wj * dirichlet(ax, n) * dirichlet(ay, n);
  }
  kern[idx] = (float)(acc / ((double)n * n));
}

// Direct non-uniform DFT of the coil images (data generation and A^H b are
// set-up work, off the iteration): FP64 phases and sums.
//   forward: kdata[s][c][j] = (1/n) sum_(y,x) S_c x [y][x] exp(-2 pi i (kx_j x + ky_j y)/n)
//   adjoint: y[s][r]        = sum_c conj(S_c[r]) (1/n) sum_j kdata[s][c][j] exp(+2 pi i k_j.r/n)
__global__ __launch_bounds__(256) void k_nudft_forward(const float2 *__restrict__ sens, const float2 *__restrict__ x,
                                                       const float *__restrict__ traj, int J, int n, int C,
                                                       int slices, float2 *__restrict__ kdata) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)slices * C * J) return;
  const int j = (int)(idx % J);
  const int sc = (int)(idx / J);
  const int s = sc / C;
  const double kx = traj[((size_t)s * J + j) * 2], ky = traj[((size_t)s * J + j) * 2 + 1];
  const float2 *sm = sens + (size_t)sc * n * n;
  const float2 *xs = x + (size_t)s * n * n;
  // exp(-2 pi i kx / n) and exp(-2 pi i ky / n): the per-pixel phase advances by rotation
  const double wxr = cos(-2.0 * M_PI * kx / n), wxi = sin(-2.0 * M_PI * kx / n);
  double ar = 0.0, ai = 0.0;
  for (int yy = 0; yy < n; ++yy) {
    double pr = cos(-2.0 * M_PI * ky * yy / n), pi_ = sin(-2.0 * M_PI * ky * yy / n);
    double rr = 0.0, ri = 0.0;
    for (int xx = 0; xx < n; ++xx) {
      const float2 a = sm[(size_t)yy * n + xx], b = xs[(size_t)yy * n + xx];
      const double ur = (double)a.x * b.x - (double)a.y * b.y, ui = (double)a.x * b.y + (double)a.y * b.x;
      rr += ur * pr - ui * pi_;
      ri += ur * pi_ + ui * pr;
      const double npr = pr * wxr - pi_ * wxi;
      pi_ = pr * wxi + pi_ * wxr;
      pr = npr;
    }
    ar += rr;
    ai += ri;
  }
  kdata[idx] = make_float2((float)(ar / n), (float)(ai / n));
}

__global__ __launch_bounds__(256) void k_nudft_adjoint(const float2 *__restrict__ sens,
                                                       const float2 *__restrict__ kdata,
                                                       const float *__restrict__ traj, int J, int n, int C,
                                                       int slices, float2 *__restrict__ y) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)slices * n * n) return;
  const int s = (int)(idx / ((size_t)n * n));
  const int r = (int)(idx % ((size_t)n * n));
  const int yy = r / n, xx = r % n;
  const float *ts = traj + (size_t)s * J * 2;
  double outr = 0.0, outi = 0.0;
  // four coils per sweep over the samples share each sample's phase factor
  for (int c0 = 0; c0 < C; c0 += 4) {
    double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < J; ++j) {
      // phase (kx x + ky y)/n in cycles, reduced to [-1/2, 1/2] in FP64 before the sine
      double ph = ((double)ts[2 * j] * xx + (double)ts[2 * j + 1] * yy) / n;
      ph -= rint(ph);
      float sn, cs;
      sincosf((float)(2.0 * M_PI * ph), &sn, &cs);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (c0 + q < C) {
          const float2 b = kdata[((size_t)s * C + c0 + q) * J + j];
          ar[q] += (double)b.x * cs - (double)b.y * sn;
          ai[q] += (double)b.x * sn + (double)b.y * cs;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (c0 + q < C) {
        const float2 sm = sens[((size_t)s * C + c0 + q) * n * n + r];
        outr += sm.x * ar[q] + sm.y * ai[q];
        outi += sm.x * ai[q] - sm.y * ar[q];
      }
    }
  }
  y[idx] = make_float2((float)(outr / n), (float)(outi / n));
}

// ---------------------------------------------------------------------------
// Packed coil maps of the phase-encode operator.  In the natural layout one load
// instruction of a k_normal_1d wave touches T rows and only CPW * 8 bytes of each
// (the wave holds CPW columns: 32 rows x 16 bytes at N = 384), which keeps the
// texture address unit busy; the packed layout stores, per slice, the values in
// the order the kernel's lanes consume them: [column block][coil][wave][pair p]
// [lane][h], where lane l's element i = 2p + h is its natural value at row pos_i
// (every slot holds a value: these plans have one input block of T rows).  A
// wave then reads one coil's pair p as 1 KB of contiguous bytes (64 lanes x 16
// bytes).  Same size as the natural layout.
template <int N> struct Pack1D {
  using Gm = Geo1D<N>;
  using F = typename Gm::F;
  static constexpr int PI = Gm::P_IN;
  static constexpr int W = Gm::THREADS / 64;
  static_assert(PI % 2 == 0, "packed pairs need an even value count per lane");
  static constexpr int PAIRS = PI / 2;
  static constexpr unsigned PAIR_BYTES = 64u * 16u;                 // one pair of a wave
  static constexpr unsigned COIL_BYTES = (unsigned)W * PAIRS * PAIR_BYTES;   // one coil of a block
};

// natural -> packed.  Block = one (column block, coil, slice): it reads the
// block's COLS columns of every row (whole 128-byte row segments), places each
// value at its packed position in LDS, and writes the block's packed run of
// COLS * N values contiguously.  Every plan of this operator has one input
// register block (NB_in = 1) with T == B_in, so row y is element i = y / T of
// lane row j0 = y % T and no packed slot is padding.
template <int N>
__global__ __launch_bounds__(256) void k_pack_1d(const float2 *__restrict__ sens, float2 *__restrict__ out, int C) {
  using P = Pack1D<N>;
  using Gm = typename P::Gm;
  using F = typename P::F;
  static_assert(F::NB_in == 1 && F::T == F::B_in, "packed order assumes one input block of T rows");
  constexpr int COLS = Gm::COLS, RUN = COLS * N;
  static_assert(RUN * (int)sizeof(float2) <= 65536, "one block's run must fit the workgroup's LDS");
  __shared__ float2 s_run[RUN];
  const int bx = blockIdx.x, c = blockIdx.y, s = blockIdx.z;
  const float2 *src = sens + ((size_t)s * C + c) * N * N + (size_t)bx * COLS;
  for (int e = threadIdx.x; e < RUN; e += 256) {
    const int y = e / COLS, cl = e % COLS;
    const int wv = cl / Gm::CPW, ci = cl % Gm::CPW;
    const int j0 = y % F::T, i = y / F::T;
    const int ln = j0 * Gm::CPW + ci;
    s_run[((wv * P::PAIRS + i / 2) * 64 + ln) * 2 + (i % 2)] = src[(size_t)y * N + cl];
  }
  __syncthreads();
  float2 *dst = out + (size_t)s * C * N * N + ((size_t)bx * C + c) * RUN;
  for (int e = threadIdx.x; e < RUN; e += 256) dst[e] = s_run[e];
}

// ---------------------------------------------------------------------------
// One-pass normal operator for a phase-encode mask (sampled rows ky, all kx):
// F^H M F = (F_y^H M_y F_y) (x) I, so each column only needs a y transform pair.
// Block = COLS columns of one slice, wave-private transform groups; all coils
// are accumulated in registers; the next coil map is loaded while the current
// one is transformed (packed) or after it has been combined (natural).  PACKED:
// `sens` is in the packed layout above (same arithmetic, so bitwise the same
// result).
// The per-lane index math of the transforms stays in registers across the coil
// loop (the compiler hoists it; recomputing it for every coil costs more).
template <int N, bool PACKED>
__global__ __launch_bounds__(Geo1D<N>::THREADS, 2) void k_normal_1d(const float2 *__restrict__ x,
                                                   const float2 *__restrict__ sens,
                                                   const uint8_t *__restrict__ mask,
                                                   float2 *__restrict__ y, const float2 *w, float alpha,
                                                   float beta, int C, int *k_inc) {
  using Gm = Geo1D<N>;
  if (k_inc && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *k_inc += 1;
  using F = typename Gm::F;
  using I = typename Gm::I;
  constexpr int T = Gm::T;
  constexpr int PI = Gm::P_IN;
  __shared__ float2 s_twF[TwLayout<F>::size()];
  __shared__ float2 s_twI[TwLayout<I>::size()];
  __shared__ float2 s_buf[Gm::COLS * Gm::LDSN];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int ci = ln % Gm::CPW, col = wv * Gm::CPW + ci, j0 = ln / Gm::CPW;
  const int kx = blockIdx.x * Gm::COLS + col;
  const int s = blockIdx.y;
  const uint8_t *mask_s = mask + (size_t)s * N;
  const float2 *xs = x + (size_t)s * N * N;
  const float2 *ss = sens + (size_t)s * C * N * N;
  // buffer resource over this slice's coil maps (raw, byte-addressed; reads past
  // the end return zero)
  const __amdgpu_buffer_rsrc_t srsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2 *>(ss), (short)0, C * N * N * (int)sizeof(float2), 0x00020000);
  // positions yy = j + r * F::B_in (F input layout == I output layout)
  auto pos = [&](int i) { return (j0 + (i / F::R_in) * T + (i % F::R_in) * F::B_in) * N + kx; };
  auto okp = [&](int i) { return lay_in_ok<F>(j0 + (i / F::R_in) * T); };
  unsigned mbits = 0;
#pragma unroll
  for (int b = 0; b < F::NB_out; ++b) {
    const int j = j0 + b * T;
#pragma unroll
    for (int r = 0; r < F::R_out; ++r)
      if (lay_out_ok<F>(j) && mask_s[j + r * F::B_out] != 0) mbits |= 1u << (b * F::R_out + r);
  }
  // packed: the next coil's maps go to `sn` between the forward and the inverse
  // transform (contiguous loads leave the texture unit free enough for that
  // overlap; natural-layout loads wait until the combine is done)
  float2 xv[PI], acc[PI], sc[PI], sn[PACKED ? PI : 1];
  // packed: this lane's first pair within coil 0 of its block; a coil adds a
  // scalar offset, a pair a constant one
  using Pk = Pack1D<N>;
  const unsigned lane_off =
      PACKED ? ((((unsigned)blockIdx.x * C * Pk::W + wv) * Pk::PAIRS) * 64u + ln) * 16u : 0u;
  auto load_packed = [&](float2 *dst, int c) {
#pragma unroll
    for (int p = 0; p < Pk::PAIRS; ++p) {
      const float4 f = __builtin_bit_cast(
          float4, __builtin_amdgcn_raw_buffer_load_b128(srsrc, lane_off + p * Pk::PAIR_BYTES,
                                                        (int)(c * Pk::COIL_BYTES), 0));
      dst[2 * p] = make_float2(f.x, f.y);
      dst[2 * p + 1] = make_float2(f.z, f.w);
    }
  };
#pragma unroll
  for (int i = 0; i < PI; ++i) {
    xv[i] = okp(i) ? xs[pos(i)] : make_float2(0.f, 0.f);
    if constexpr (!PACKED) sc[i] = okp(i) ? ss[pos(i)] : make_float2(0.f, 0.f);
    acc[i] = make_float2(0.f, 0.f);
  }
  if constexpr (PACKED) load_packed(sc, 0);
  load_tw(s_twF, TwBase<N>::v + TwBlock<N>::f1, TwLayout<F>::size());
  load_tw(s_twI, TwBase<N>::v + TwBlock<N>::i1, TwLayout<I>::size());
  __syncthreads();
  for (int c = 0; c < C; ++c) {
    float2 v[Gm::P];
#pragma unroll
    for (int i = 0; i < PI; ++i) v[i] = cmul(sc[i], xv[i]);
    const int jl = j0;
    float2 *bl = s_buf + wv * Gm::CPW * Gm::LDSN + ci;

    fft_run<F, -1, Gm::CPW>(v, bl, jl, s_twF);
#pragma unroll
    for (int i = 0; i < Gm::P_OUT; ++i)
      if (!((mbits >> i) & 1u)) v[i] = make_float2(0.f, 0.f);
    if constexpr (PACKED) {
      if (c + 1 < C) load_packed(sn, c + 1);
    }
    fft_run<I, +1, Gm::CPW>(v, bl, jl, s_twI);
#pragma unroll
    for (int i = 0; i < PI; ++i) acc[i] = cadd(acc[i], cmulc(v[i], sc[i]));
    if constexpr (PACKED) {
#pragma unroll
      for (int i = 0; i < PI; ++i) sc[i] = sn[i];
    } else if (c + 1 < C) {
      // the next coil map through buffer loads: the per-lane byte offsets are the
      // same for every coil and the coil's offset is a scalar, so the loop does no
      // 64-bit address arithmetic per load
      const int soff = (c + 1) * N * N * (int)sizeof(float2);
#pragma unroll
      for (int i = 0; i < PI; ++i) {
        const unsigned o = (unsigned)((j0 + (i / F::R_in) * T + (i % F::R_in) * F::B_in) * N + kx) * 8u;
        sc[i] = okp(i) ? __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(srsrc, o, soff, 0))
                       : make_float2(0.f, 0.f);
      }
    }
  }
  float2 *ys = y + (size_t)s * N * N;
  const float2 *ws = w ? w + (size_t)s * N * N : nullptr;
  if constexpr (PACKED) {
    // the block's outputs go through LDS so that y is written in whole row
    // segments (a wave instruction covers four rows of the block's COLS
    // columns) rather than 16 bytes of a row per wave, which let partly written
    // lines leave the L2 early and be written twice
    constexpr int TS = Gm::COLS + 1;   // padded tile row
    static_assert(N * TS <= Gm::COLS * Gm::LDSN, "output tile fits the exchange buffer");
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PI; ++i) {
      if (okp(i)) {
        float2 out = cscale(acc[i], alpha);
        if (ws) out = cadd(out, cscale(ws[pos(i)], beta));
        s_buf[(j0 + (i / F::R_in) * T + (i % F::R_in) * F::B_in) * TS + col] = out;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * Gm::COLS; e += Gm::THREADS) {
      const int row = e / Gm::COLS, c = e % Gm::COLS;
      ys[(size_t)row * N + blockIdx.x * Gm::COLS + c] = s_buf[row * TS + c];
    }
  } else {
#pragma unroll
    for (int i = 0; i < PI; ++i) {
      if (okp(i)) {
        float2 out = cscale(acc[i], alpha);
        if (ws) out = cadd(out, cscale(ws[pos(i)], beta));
        ys[pos(i)] = out;
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
// Complex soft-threshold, branch-free: keep |w| > lam as |w|^2 > lam^2 and scale
// by 1 - lam / |w| with the hardware reciprocal square root (about 1 ulp); adds
// |soft(w)| = |w| - lam to l1.  w = 0 gives exactly 0 for any lam >= 0.
__device__ __forceinline__ float2 soft_thr(float2 w, float lam, float &l1) {
  const float m2 = w.x * w.x + w.y * w.y;
  const bool keep = m2 > lam * lam;
  const float r = __builtin_amdgcn_rsqf(keep ? m2 : 1.0f);
  const float sc = keep ? 1.0f - lam * r : 0.0f;
  l1 += keep ? m2 * r - lam : 0.0f;
  return make_float2(w.x * sc, w.y * sc);
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

// Levels l >= 2 of the Haar prox, one lane group of stride 2^(l-2) at a time:
// gather the group's four LL values, threshold its three detail coefficients
// (and the final LL at the last level), recurse to the next level, then invert
// this level and keep the value at this lane's position.  Compile-time recursion
// keeps every coefficient in registers.
__device__ __forceinline__ float2 pick4(int bx, int by, float2 a, float2 b, float2 c, float2 d) {
  const float2 top = bx ? b : a, bot = bx ? d : c;
  return by ? bot : top;
}

template <int L, int LEVELS>
__device__ __forceinline__ float2 haar_levels(float2 ll, int tx, int ty, float lam, float &l1) {
  if constexpr (L > LEVELS) {
    return ll;
  } else {
    constexpr int st = 1 << (L - 2);
    const int bx = (tx >> (L - 2)) & 1, by = (ty >> (L - 2)) & 1;
    const float2 ox = shfl_xor2(ll, st), oy = shfl_xor2(ll, 8 * st), od = shfl_xor2(ll, 9 * st);
    // the group's 2 x 2 block [[A, B], [C, D]] seen from this lane's corner
    const float2 A = pick4(bx, by, ll, ox, oy, od);
    const float2 B = pick4(bx, by, ox, ll, od, oy);
    const float2 Cc = pick4(bx, by, oy, od, ll, ox);
    const float2 D = pick4(bx, by, od, oy, ox, ll);
    Quad r = haar4(A, B, Cc, D);
    float l1g = 0.f;   // identical in the four lanes of the group: count it once
    r.dx = soft_thr(r.dx, lam, l1g);
    r.dy = soft_thr(r.dy, lam, l1g);
    r.dd = soft_thr(r.dd, lam, l1g);
    if constexpr (L == LEVELS) r.ll = soft_thr(r.ll, lam, l1g);
    if (!(tx & (2 * st - 1)) && !(ty & (2 * st - 1))) l1 += l1g;
    r.ll = haar_levels<L + 1, LEVELS>(r.ll, tx, ty, lam, l1);
    float2 a, b, c, d;
    ihaar4(r, a, b, c, d);
    return pick4(bx, by, a, b, c, d);
  }
}

template <int LEVELS>
__global__ __launch_bounds__(64) void k_step(const float2 *__restrict__ z, const float2 *__restrict__ pg,
                                             const float2 *x_old, float2 *x_new, float2 *z_new,
                                             float pg_scale, float lam_arg, float beta_arg,
                                             const int *__restrict__ k_dev, int use_k, int N,
                                             double *__restrict__ partials,
                                             const float *__restrict__ lam_s) {
  const int lane = threadIdx.x, tx = lane & 7, ty = lane >> 3;
  // tiles numbered over all slices like the row passes' blocks (xcd_block)
  const int ntile = gridDim.x * gridDim.y;
  const int tg = xcd_block((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x, ntile * gridDim.z);
  const int s = tg / ntile, tl = tg % ntile;
  // per-slice threshold when a table is given
  const float lam = lam_s ? lam_s[s] : lam_arg;
  const int px = (tl % gridDim.x) * 16 + 2 * tx, py = (tl / gridDim.x) * 16 + 2 * ty;
  const size_t o0 = (size_t)s * N * N + (size_t)py * N + px, o1 = o0 + N;
  // unconditional scalar load: its latency overlaps the vector loads below
  const int kk = *k_dev;
  const float4 z0 = *reinterpret_cast<const float4 *>(z + o0), z1 = *reinterpret_cast<const float4 *>(z + o1);
  const float4 g0 = *reinterpret_cast<const float4 *>(pg + o0), g1 = *reinterpret_cast<const float4 *>(pg + o1);
  const float4 q0 = *reinterpret_cast<const float4 *>(x_old + o0), q1 = *reinterpret_cast<const float4 *>(x_old + o1);
  const float2 a = make_float2(z0.x - pg_scale * g0.x, z0.y - pg_scale * g0.y);
  const float2 b = make_float2(z0.z - pg_scale * g0.z, z0.w - pg_scale * g0.w);
  const float2 c = make_float2(z1.x - pg_scale * g1.x, z1.y - pg_scale * g1.y);
  const float2 d = make_float2(z1.z - pg_scale * g1.z, z1.w - pg_scale * g1.w);
  float l1 = 0.f;
  Quad q = haar4(a, b, c, d);
  q.dx = soft_thr(q.dx, lam, l1);
  q.dy = soft_thr(q.dy, lam, l1);
  q.dd = soft_thr(q.dd, lam, l1);
  if constexpr (LEVELS == 1) q.ll = soft_thr(q.ll, lam, l1);
  q.ll = haar_levels<2, LEVELS>(q.ll, tx, ty, lam, l1);
  float2 na, nb, nc, nd;
  ihaar4(q, na, nb, nc, nd);
  const float2 oa = make_float2(q0.x, q0.y), ob = make_float2(q0.z, q0.w);
  const float2 oc = make_float2(q1.x, q1.y), od = make_float2(q1.z, q1.w);
  float dx2 = 0.f, xn2 = 0.f;
  auto acc = [&](float2 n, float2 o) {
    const float ex = n.x - o.x, ey = n.y - o.y;
    dx2 += ex * ex + ey * ey;
    xn2 += n.x * n.x + n.y * n.y;
  };
  acc(na, oa); acc(nb, ob); acc(nc, oc); acc(nd, od);
  const float beta = use_k ? (float)((double)kk / ((double)kk + 3.0)) : beta_arg;
  auto mom = [&](float2 n, float2 o) {
    return make_float2(n.x + beta * (n.x - o.x), n.y + beta * (n.y - o.y));
  };
  const float2 za = mom(na, oa), zb = mom(nb, ob), zc = mom(nc, oc), zd = mom(nd, od);
  *reinterpret_cast<float4 *>(x_new + o0) = make_float4(na.x, na.y, nb.x, nb.y);
  *reinterpret_cast<float4 *>(x_new + o1) = make_float4(nc.x, nc.y, nd.x, nd.y);
  *reinterpret_cast<float4 *>(z_new + o0) = make_float4(za.x, za.y, zb.x, zb.y);
  *reinterpret_cast<float4 *>(z_new + o1) = make_float4(zc.x, zc.y, zd.x, zd.y);
  // per-lane sums (a few FP32 terms each) widen to FP64 for the wave and grid sums
  const double l1d = wave_sum((double)l1), dx2d = wave_sum((double)dx2), xn2d = wave_sum((double)xn2);
  if (lane == 0) {
    const size_t blk = (size_t)tg;   // partial sums in tile order, whatever the block order
    partials[3 * blk + 0] = l1d;
    partials[3 * blk + 1] = dx2d;
    partials[3 * blk + 2] = xn2d;
  }
}

// ---------------------------------------------------------------------------
// Reverse mode of the prox step (the backward pass through unrolled iterations).
// Complex cotangents are real gradients packed as complex numbers.
// Pull-back of w = soft(u, lam) at u for the cotangent wb: on the support the
// Jacobian (a map of R^2) keeps the direction u/|u| with factor 1 and scales the
// perpendicular one by 1 - lam/|u|; dw/dlam = -u/|u| (accumulated in lb).
__device__ __forceinline__ float2 soft_vjp(float2 u, float2 wb, float lam, float &lb) {
  const float m2 = u.x * u.x + u.y * u.y;
  const bool keep = m2 > lam * lam;
  const float r = __builtin_amdgcn_rsqf(keep ? m2 : 1.0f);
  const float ux = u.x * r, uy = u.y * r;
  const float rad = ux * wb.x + uy * wb.y;
  const float f = 1.0f - lam * r;
  lb += keep ? -rad : 0.0f;
  const float bx = rad * ux + f * (wb.x - rad * ux), by = rad * uy + f * (wb.y - rad * uy);
  return keep ? make_float2(bx, by) : make_float2(0.f, 0.f);
}

// Levels l >= 2 of the pull-back, mirroring haar_levels: the group's analysis
// of v (u) and of the cotangent (wb) side by side; returns this lane's LL
// cotangent of level l - 1.
template <int L, int LEVELS>
__device__ __forceinline__ float2 haar_vjp_levels(float2 llu, float2 llw, int tx, int ty, float lam, float &lb) {
  constexpr int st = 1 << (L - 2);
  const int bx = (tx >> (L - 2)) & 1, by = (ty >> (L - 2)) & 1;
  const float2 ux = shfl_xor2(llu, st), uy = shfl_xor2(llu, 8 * st), ud = shfl_xor2(llu, 9 * st);
  const float2 wx = shfl_xor2(llw, st), wy = shfl_xor2(llw, 8 * st), wd = shfl_xor2(llw, 9 * st);
  const Quad ru = haar4(pick4(bx, by, llu, ux, uy, ud), pick4(bx, by, ux, llu, ud, uy),
                        pick4(bx, by, uy, ud, llu, ux), pick4(bx, by, ud, uy, ux, llu));
  const Quad rw = haar4(pick4(bx, by, llw, wx, wy, wd), pick4(bx, by, wx, llw, wd, wy),
                        pick4(bx, by, wy, wd, llw, wx), pick4(bx, by, wd, wy, wx, llw));
  float lg = 0.f;   // identical in the four lanes of the group: counted once
  Quad rb;
  rb.dx = soft_vjp(ru.dx, rw.dx, lam, lg);
  rb.dy = soft_vjp(ru.dy, rw.dy, lam, lg);
  rb.dd = soft_vjp(ru.dd, rw.dd, lam, lg);
  if constexpr (L == LEVELS) {
    rb.ll = soft_vjp(ru.ll, rw.ll, lam, lg);
  } else {
    rb.ll = haar_vjp_levels<L + 1, LEVELS>(ru.ll, rw.ll, tx, ty, lam, lb);
  }
  if (!(tx & (2 * st - 1)) && !(ty & (2 * st - 1))) lb += lg;
  float2 a, b, c, d;
  ihaar4(rb, a, b, c, d);
  return pick4(bx, by, a, b, c, d);
}

// Pull-back of one step x_(k+1) = prox(z_k - pg_k), z_(k+1) = (1 + beta) x_(k+1)
// - beta x_k, given xb = x_bar_(k+1) and zb = z_bar_(k+1):
//   vb = Psi^H J_soft(Psi v)^T Psi (xb + (1 + beta) zb),   v = z - pg,
//   xb <- -beta zb  (x_bar_k, in place), FP64 partial sums of lambda_bar.
template <int LEVELS>
__global__ __launch_bounds__(64) void k_prox_vjp(const float2 *__restrict__ z, const float2 *__restrict__ pg,
                                                 float2 *xb, const float2 *__restrict__ zb,
                                                 float2 *__restrict__ vb, float lam, float beta, int N,
                                                 double *__restrict__ partials) {
  const int lane = threadIdx.x, tx = lane & 7, ty = lane >> 3;
  const int s = blockIdx.z;
  const int px = blockIdx.x * 16 + 2 * tx, py = blockIdx.y * 16 + 2 * ty;
  const size_t o0 = (size_t)s * N * N + (size_t)py * N + px, o1 = o0 + N;
  auto ld = [](const float2 *p, size_t o) { return *reinterpret_cast<const float4 *>(p + o); };
  const float4 z0 = ld(z, o0), z1 = ld(z, o1), g0 = ld(pg, o0), g1 = ld(pg, o1);
  const float4 x0 = ld(xb, o0), x1 = ld(xb, o1), q0 = ld(zb, o0), q1 = ld(zb, o1);
  const float bz = 1.0f + beta;
  const float2 va = make_float2(z0.x - g0.x, z0.y - g0.y), vbb = make_float2(z0.z - g0.z, z0.w - g0.w);
  const float2 vc = make_float2(z1.x - g1.x, z1.y - g1.y), vd = make_float2(z1.z - g1.z, z1.w - g1.w);
  const float2 wa = make_float2(x0.x + bz * q0.x, x0.y + bz * q0.y), wb = make_float2(x0.z + bz * q0.z, x0.w + bz * q0.w);
  const float2 wc = make_float2(x1.x + bz * q1.x, x1.y + bz * q1.y), wd = make_float2(x1.z + bz * q1.z, x1.w + bz * q1.w);
  const Quad qu = haar4(va, vbb, vc, vd), qw = haar4(wa, wb, wc, wd);
  float lb = 0.f;
  Quad rb;
  rb.dx = soft_vjp(qu.dx, qw.dx, lam, lb);
  rb.dy = soft_vjp(qu.dy, qw.dy, lam, lb);
  rb.dd = soft_vjp(qu.dd, qw.dd, lam, lb);
  if constexpr (LEVELS == 1) {
    rb.ll = soft_vjp(qu.ll, qw.ll, lam, lb);
  } else {
    rb.ll = haar_vjp_levels<2, LEVELS>(qu.ll, qw.ll, tx, ty, lam, lb);
  }
  float2 ra, rbv, rc, rd;
  ihaar4(rb, ra, rbv, rc, rd);
  *reinterpret_cast<float4 *>(vb + o0) = make_float4(ra.x, ra.y, rbv.x, rbv.y);
  *reinterpret_cast<float4 *>(vb + o1) = make_float4(rc.x, rc.y, rd.x, rd.y);
  *reinterpret_cast<float4 *>(xb + o0) = make_float4(-beta * q0.x, -beta * q0.y, -beta * q0.z, -beta * q0.w);
  *reinterpret_cast<float4 *>(xb + o1) = make_float4(-beta * q1.x, -beta * q1.y, -beta * q1.z, -beta * q1.w);
  const double l = wave_sum((double)lb);
  if (lane == 0) partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = l;
}

// pv = sum_i c_i q_i over the d + 1 images q_i = q + i * n (q_0 = v_bar, q_i =
// N'^i v_bar) and FP64 partial sums of Re <q_i, g>, (d + 1) per block.
struct CoefArg { float c[9]; };
__global__ __launch_bounds__(256) void k_poly_combine_dot(const float2 *__restrict__ q, int terms, size_t n,
                                                          const float2 *__restrict__ g, CoefArg c,
                                                          float2 *__restrict__ pv, double *__restrict__ partials) {
  __shared__ double s_red[4][9];
  double dot[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) dot[i] = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const float2 gv = g[e];
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (i < terms) {
        const float2 qi = q[(size_t)i * n + e];
        acc.x += c.c[i] * qi.x;
        acc.y += c.c[i] * qi.y;
        dot[i] += (double)qi.x * gv.x + (double)qi.y * gv.y;
      }
    }
    pv[e] = acc;
  }
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if (i < terms) {
      const double v = wave_sum_d(dot[i]);
      if (ln == 0) s_red[wv][i] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < terms)
    partials[(size_t)blockIdx.x * terms + threadIdx.x] =
        ((s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) + s_red[2][threadIdx.x]) + s_red[3][threadIdx.x];
}

// out[c] += scale * sum_i partials[i * width + c] for c < width <= 16, one wave,
// fixed order
__global__ __launch_bounds__(64) void k_reduce_add(const double *__restrict__ partials, int count, int width,
                                                   double scale, double *__restrict__ out) {
  for (int c = 0; c < width && c < 16; ++c) {
    double a = 0.0;
    for (int i = threadIdx.x; i < count; i += 64) a += partials[(size_t)i * width + c];
    a = wave_sum_d(a);
    if (threadIdx.x == 0) out[c] += scale * a;
  }
}

// ---------------------------------------------------------------------------
// Small helpers
// Sum `width`-strided FP64 partials (width <= 4) in a fixed order into
// out[0..width) with one wave: lane-strided sums, then a fixed butterfly.  If
// k_dev is given, also advances the solver's device iteration counter.
__global__ __launch_bounds__(64) void k_reduce(const double *__restrict__ partials, int count, int width,
                                               double *__restrict__ out, int *k_dev) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < count; i += 64)
    for (int c = 0; c < width && c < 4; ++c) a[c] += partials[(size_t)i * width + c];
  for (int c = 0; c < width && c < 4; ++c) {
    const double v = wave_sum_d(a[c]);
    if (threadIdx.x == 0) out[c] = v;
  }
  if (threadIdx.x == 0 && k_dev) *k_dev = *k_dev + 1;
}

// Per-segment version of k_reduce, one wave per segment (blockIdx.x): segment s
// covers partials [cb[s] * len, cb[s+1] * len) if cb is given, else
// [s * len, (s+1) * len), in units of `width`-tuples; out[s * width + c].
__global__ __launch_bounds__(64) void k_reduce_seg(const double *__restrict__ partials,
                                                   const int *__restrict__ cb, int len, int width,
                                                   double *__restrict__ out) {
  const int s = blockIdx.x;
  const int b = cb ? cb[s] * len : s * len;
  const int e = cb ? cb[s + 1] * len : (s + 1) * len;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = b + threadIdx.x; i < e; i += 64)
    for (int c = 0; c < width && c < 4; ++c) a[c] += partials[(size_t)i * width + c];
  for (int c = 0; c < width && c < 4; ++c) {
    const double v = wave_sum_d(a[c]);
    if (threadIdx.x == 0) out[(size_t)s * width + c] = v;
  }
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

// FP64 partial sums of Re <x, u> and Re <x, v> (grid-stride), two per block
__global__ __launch_bounds__(256) void k_dot2(const float2 *__restrict__ x, const float2 *__restrict__ u,
                                              const float2 *__restrict__ v, size_t n, double *__restrict__ partials) {
  __shared__ double s[2][4];
  double a = 0.0, b = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float2 xe = x[i], ue = u[i], ve = v[i];
    a += (double)xe.x * ue.x + (double)xe.y * ue.y;
    b += (double)xe.x * ve.x + (double)xe.y * ve.y;
  }
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s[0][wv] = a;
    s[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x < 2)
    partials[2 * blockIdx.x + threadIdx.x] =
        ((s[threadIdx.x][0] + s[threadIdx.x][1]) + s[threadIdx.x][2]) + s[threadIdx.x][3];
}

// data term through the normal equations: out = dots[0] - 2 dots[1] + 1
__global__ void k_normal_eq_data(const double *__restrict__ dots, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = dots[0] - 2.0 * dots[1] + 1.0;
}

// the solver's iteration counter, set on the stream (no host memory involved)
__global__ void k_set_counter(int *k, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *k = v;
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
