// Register/LDS mixed-radix FFT engine for gfx950 (wave64), FP32 complex.
//
// A length-N transform is carried by T lanes of one workgroup ("FFT group").
// It runs as a Stockham auto-sort sequence of radix stages R_0, R_1, ... whose
// product is N.  Stage s (sub-transform length Ns = R_0 ... R_{s-1}) takes
// butterfly j (0 <= j < N/R) from inputs in[j + r N/R], multiplies input r by
// exp(dir 2 pi i r (j mod Ns) / (Ns R)), applies a length-R DFT in registers
// and writes output r to out[(j / Ns) Ns R + (j mod Ns) + r Ns].  The result is
// the DFT in natural order.  Lane j0 of the group owns butterflies
// j = j0 + b T, b = 0 .. ceil((N/R)/T) - 1; stages hand data over through a
// padded LDS buffer.  Consequences used by the kernels:
//   * the first stage's inputs in lane j0 are x[j0 + b T + r N/R_0], so the
//     kernels load them straight from global memory (coalesced);
//   * the last stage's outputs are X[j0 + b T + r N/R_last], stored the same way;
//   * a forward plan (R_0 .. R_L) and its mirror (R_L .. R_0) used for the
//     inverse meet in registers: the forward's outputs are exactly the
//     inverse's inputs, so forward -> k-space mask -> inverse needs no exchange.
// Transforms are unnormalised here; the kernels fold 1/N into their scalars.

#pragma once
#include <hip/hip_runtime.h>

namespace pf {

// ---------------------------------------------------------------- complex ops
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// (x + iy) * (dir i)
template <int DIR> __device__ __forceinline__ float2 mul_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// -------------------------------------------- exact-constant twiddles of small DFTs
// exp(-2 pi i m / R) rounded to FP32 (forward sign); the inverse uses the conjugate.
struct C2 { float c, s; };
template <int R> struct SmallTw;
template <> struct SmallTw<6> {
  static constexpr C2 w[6] = {{1.f, 0.f}, {5.000000000e-01f, -8.660253882e-01f},
                              {-5.000000000e-01f, -8.660253882e-01f}, {-1.f, 0.f},
                              {-5.000000000e-01f, 8.660253882e-01f}, {5.000000000e-01f, 8.660253882e-01f}};
};
template <> struct SmallTw<8> {
  static constexpr C2 w[8] = {{1.f, 0.f}, {7.071067691e-01f, -7.071067691e-01f}, {0.f, -1.f},
                              {-7.071067691e-01f, -7.071067691e-01f}, {-1.f, 0.f},
                              {-7.071067691e-01f, 7.071067691e-01f}, {0.f, 1.f},
                              {7.071067691e-01f, 7.071067691e-01f}};
};
template <> struct SmallTw<10> {
  static constexpr C2 w[10] = {{1.f, 0.f}, {8.090170026e-01f, -5.877852440e-01f},
                               {3.090170026e-01f, -9.510565400e-01f}, {-3.090170026e-01f, -9.510565400e-01f},
                               {-8.090170026e-01f, -5.877852440e-01f}, {-1.f, 0.f},
                               {-8.090170026e-01f, 5.877852440e-01f}, {-3.090170026e-01f, 9.510565400e-01f},
                               {3.090170026e-01f, 9.510565400e-01f}, {8.090170026e-01f, 5.877852440e-01f}};
};
template <> struct SmallTw<12> {
  static constexpr C2 w[12] = {{1.f, 0.f}, {8.660253882e-01f, -5.000000000e-01f},
                               {5.000000000e-01f, -8.660253882e-01f}, {0.f, -1.f},
                               {-5.000000000e-01f, -8.660253882e-01f}, {-8.660253882e-01f, -5.000000000e-01f},
                               {-1.f, 0.f}, {-8.660253882e-01f, 5.000000000e-01f},
                               {-5.000000000e-01f, 8.660253882e-01f}, {0.f, 1.f},
                               {5.000000000e-01f, 8.660253882e-01f}, {8.660253882e-01f, 5.000000000e-01f}};
};
template <> struct SmallTw<16> {
  static constexpr C2 w[16] = {{1.f, 0.f}, {9.238795042e-01f, -3.826834261e-01f},
                               {7.071067691e-01f, -7.071067691e-01f}, {3.826834261e-01f, -9.238795042e-01f},
                               {0.f, -1.f}, {-3.826834261e-01f, -9.238795042e-01f},
                               {-7.071067691e-01f, -7.071067691e-01f}, {-9.238795042e-01f, -3.826834261e-01f},
                               {-1.f, 0.f}, {-9.238795042e-01f, 3.826834261e-01f},
                               {-7.071067691e-01f, 7.071067691e-01f}, {-3.826834261e-01f, 9.238795042e-01f},
                               {0.f, 1.f}, {3.826834261e-01f, 9.238795042e-01f},
                               {7.071067691e-01f, 7.071067691e-01f}, {9.238795042e-01f, 3.826834261e-01f}};
};
template <> struct SmallTw<20> {
  static constexpr C2 w[20] = {{1.f, 0.f}, {9.510565400e-01f, -3.090170026e-01f},
                               {8.090170026e-01f, -5.877852440e-01f}, {5.877852440e-01f, -8.090170026e-01f},
                               {3.090170026e-01f, -9.510565400e-01f}, {0.f, -1.f},
                               {-3.090170026e-01f, -9.510565400e-01f}, {-5.877852440e-01f, -8.090170026e-01f},
                               {-8.090170026e-01f, -5.877852440e-01f}, {-9.510565400e-01f, -3.090170026e-01f},
                               {-1.f, 0.f}, {-9.510565400e-01f, 3.090170026e-01f},
                               {-8.090170026e-01f, 5.877852440e-01f}, {-5.877852440e-01f, 8.090170026e-01f},
                               {-3.090170026e-01f, 9.510565400e-01f}, {0.f, 1.f},
                               {3.090170026e-01f, 9.510565400e-01f}, {5.877852440e-01f, 8.090170026e-01f},
                               {8.090170026e-01f, 5.877852440e-01f}, {9.510565400e-01f, 3.090170026e-01f}};
};

// multiply by exp(dir 2 pi i m / R) with m a compile-time constant after unrolling
template <int R, int DIR> __device__ __forceinline__ float2 twiddle_small(float2 a, int m) {
  if (m == 0) return a;
  if (4 * m == R) return mul_i<DIR>(a);
  if (2 * m == R) return make_float2(-a.x, -a.y);
  if (4 * m == 3 * R) return mul_i<-DIR>(a);
  const C2 w = SmallTw<R>::w[m];
  const float ws = DIR < 0 ? w.s : -w.s;
  return make_float2(a.x * w.c - a.y * ws, a.x * ws + a.y * w.c);
}

// ------------------------------------------------------------ small DFT kernels
// In place, natural order: v[k] <- sum_n v[n] exp(dir 2 pi i n k / R).
template <int DIR> __device__ __forceinline__ void dft2(float2 *v) {
  const float2 a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <int DIR> __device__ __forceinline__ void dft3(float2 *v) {
  constexpr float kS = 8.660253882e-01f;  // sin(2 pi / 3)
  const float2 t = cadd(v[1], v[2]);
  const float2 d = csub(v[1], v[2]);
  const float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
  const float2 r = mul_i<DIR>(cscale(d, kS));
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <int DIR> __device__ __forceinline__ void dft4(float2 *v) {
  const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  const float2 t2 = cadd(v[1], v[3]), t3 = mul_i<DIR>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <int DIR> __device__ __forceinline__ void dft5(float2 *v) {
  constexpr float c1 = 3.090170026e-01f, s1 = 9.510565400e-01f;   // cos, sin (2 pi / 5)
  constexpr float c2 = -8.090170026e-01f, s2 = 5.877852440e-01f;  // cos, sin (4 pi / 5)
  const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const float2 x0 = v[0];
  const float2 a1 = make_float2(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
  const float2 a2 = make_float2(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
  const float2 b1 = mul_i<DIR>(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  const float2 b2 = mul_i<DIR>(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  v[0] = cadd(x0, cadd(t1, t2));
  v[1] = cadd(a1, b1);
  v[4] = csub(a1, b1);
  v[2] = cadd(a2, b2);
  v[3] = csub(a2, b2);
}

template <int R, int DIR> __device__ __forceinline__ void dft(float2 *v);

// Composite R = R1 R2 in registers: n = n1 + R1 n2, k = k2 + R2 k1,
// X[k2 + R2 k1] = sum_n1 W_R1^(n1 k1) W_R^(n1 k2) sum_n2 x[n1 + R1 n2] W_R2^(n2 k2).
template <int R1, int R2, int DIR> __device__ __forceinline__ void dft_split(float2 *v) {
  constexpr int R = R1 * R2;
  float2 y[R];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    float2 col[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) col[n2] = v[n1 + R1 * n2];
    dft<R2, DIR>(col);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 * R2 + k2] = twiddle_small<R, DIR>(col[k2], n1 * k2);
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    float2 row[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) row[n1] = y[n1 * R2 + k2];
    dft<R1, DIR>(row);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = row[k1];
  }
}

template <int R, int DIR> __device__ __forceinline__ void dft(float2 *v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<DIR>(v);
  } else if constexpr (R == 3) {
    dft3<DIR>(v);
  } else if constexpr (R == 4) {
    dft4<DIR>(v);
  } else if constexpr (R == 5) {
    dft5<DIR>(v);
  } else if constexpr (R == 6) {
    dft_split<3, 2, DIR>(v);
  } else if constexpr (R == 8) {
    dft_split<4, 2, DIR>(v);
  } else if constexpr (R == 10) {
    dft_split<5, 2, DIR>(v);
  } else if constexpr (R == 12) {
    dft_split<3, 4, DIR>(v);
  } else if constexpr (R == 16) {
    dft_split<4, 4, DIR>(v);
  } else if constexpr (R == 20) {
    dft_split<5, 4, DIR>(v);
  } else {
    static_assert(R == 0, "unsupported radix");
  }
}

// ------------------------------------------- butterflies on twiddled inputs
// A stage with Ns > 1 multiplies inputs 1..R-1 of each butterfly by twiddles and
// then takes a length-R DFT whose first operations are sums and differences of
// input pairs.  For a pair (a, w b) both results come from one product folded
// into FMAs: s = a + w b (four FMAs) and a - w b = 2 a - s (two FMAs), six
// operations where the separate product, sum and difference take eight.
__device__ __forceinline__ void bfly_tw(float2 &a, float2 &b, float2 w) {
  float2 s;
  s.x = __builtin_fmaf(w.x, b.x, a.x);
  s.x = __builtin_fmaf(-w.y, b.y, s.x);
  s.y = __builtin_fmaf(w.x, b.y, a.y);
  s.y = __builtin_fmaf(w.y, b.x, s.y);
  b = make_float2(__builtin_fmaf(2.f, a.x, -s.x), __builtin_fmaf(2.f, a.y, -s.y));
  a = s;
}

// length-R2 DFT (R2 = 2 or 4) of c[n] w[n], with w[0] = 1 unless TW0
template <int R2, int DIR, bool TW0>
__device__ __forceinline__ void dft_in_tw(float2 *c, const float2 *w) {
  static_assert(R2 == 2 || R2 == 4, "twiddled inner DFTs of length 2 or 4");
  if constexpr (R2 == 2) {
    if constexpr (TW0) c[0] = cmul(c[0], w[0]);
    bfly_tw(c[0], c[1], w[1]);
  } else {
    float2 a0 = c[0], a2 = c[2], u1 = cmul(c[1], w[1]), a3 = c[3];
    if constexpr (TW0) a0 = cmul(a0, w[0]);
    bfly_tw(a0, a2, w[2]);            // a0 = t0 = x0 + x2, a2 = t1 = x0 - x2
    bfly_tw(u1, a3, w[3]);            // u1 = t2 = x1 + x3, a3 = x1 - x3
    const float2 t3 = mul_i<DIR>(a3);
    c[0] = cadd(a0, u1);
    c[2] = csub(a0, u1);
    c[1] = cadd(a2, t3);
    c[3] = csub(a2, t3);
  }
}

// length-R DFT of v[r] w_r with w_0 = 1 and w_r = w[r - 1] (the twiddles of a stage)
template <int R1, int R2, int DIR>
__device__ __forceinline__ void dft_split_tw(float2 *v, const float2 *w) {
  constexpr int R = R1 * R2;
  float2 y[R];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    float2 col[R2], wc[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      col[n2] = v[n1 + R1 * n2];
      wc[n2] = (n1 + R1 * n2) ? w[n1 + R1 * n2 - 1] : make_float2(1.f, 0.f);
    }
    if (n1 == 0)
      dft_in_tw<R2, DIR, false>(col, wc);
    else
      dft_in_tw<R2, DIR, true>(col, wc);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 * R2 + k2] = twiddle_small<R, DIR>(col[k2], n1 * k2);
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    float2 row[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) row[n1] = y[n1 * R2 + k2];
    dft<R1, DIR>(row);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = row[k1];
  }
}

template <int R, int DIR> __device__ __forceinline__ void dft_tw(float2 *v, const float2 *w) {
  if constexpr (R == 2) {
    bfly_tw(v[0], v[1], w[0]);
  } else if constexpr (R == 4) {
    const float2 w4[4] = {make_float2(1.f, 0.f), w[0], w[1], w[2]};
    dft_in_tw<4, DIR, false>(v, w4);
  } else if constexpr (R == 6) {
    dft_split_tw<3, 2, DIR>(v, w);
  } else if constexpr (R == 8) {
    dft_split_tw<4, 2, DIR>(v, w);
  } else if constexpr (R == 10) {
    dft_split_tw<5, 2, DIR>(v, w);
  } else if constexpr (R == 12) {
    dft_split_tw<3, 4, DIR>(v, w);
  } else if constexpr (R == 16) {
    dft_split_tw<4, 4, DIR>(v, w);
  } else if constexpr (R == 20) {
    dft_split_tw<5, 4, DIR>(v, w);
  } else {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r - 1]);
    dft<R, DIR>(v);
  }
}

// ------------------------------------------------------------------ plans
// Radix list (forward order); the inverse runs the mirrored list.
template <int N_, int T_, int... Rs> struct Plan {
  static constexpr int N = N_;
  static constexpr int T = T_;
  static constexpr int NST = sizeof...(Rs);
  static constexpr int R[NST] = {Rs...};
  static constexpr int ns(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= R[i];
    return p;
  }
  static constexpr int nb(int s) { return (N / R[s] + T - 1) / T; }
  static constexpr int pmax() {
    int m = 0;
    for (int s = 0; s < NST; ++s) m = (nb(s) * R[s] > m) ? nb(s) * R[s] : m;
    return m;
  }
  static constexpr int prod() {
    int p = 1;
    for (int s = 0; s < NST; ++s) p *= R[s];
    return p;
  }
  static_assert(prod() == N, "radices must multiply to N");
  // first-stage (input) and last-stage (output) register layouts
  static constexpr int R_in = R[0];
  static constexpr int R_out = R[NST - 1];
  static constexpr int B_in = N / R[0];
  static constexpr int B_out = N / R[NST - 1];
  static constexpr int NB_in = nb(0);
  static constexpr int NB_out = nb(NST - 1);
};

// padded LDS index: one spare complex every 16 breaks power-of-two bank strides
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
template <int N> struct LdsLen { static constexpr int value = N + N / 16; };

// ------------------------------------------------------------------ twiddles
// Stage s (with Ns > 1) multiplies input r of butterfly j by
// exp(-2 pi i r k / (Ns R)), k = j mod Ns.  The plan's table stores these as
// [stage][k][r-1]: the lanes of one instruction (consecutive k) then read at
// the odd-ish stride R-1, which spreads them over the LDS banks, and one lane's
// R-1 factors are contiguous.  Forward sign; the inverse conjugates on use.
template <class PL> struct TwLayout {
  static constexpr int off(int s) {
    int o = 0;
    for (int i = 0; i < s; ++i)
      if (PL::ns(i) > 1) o += PL::ns(i) * (PL::R[i] - 1);
    return o;
  }
  static constexpr int size() { return off(PL::NST) > 0 ? off(PL::NST) : 1; }
};

// ------------------------------------------------------------------ stages
template <class PL, int S, int DIR>
__device__ __forceinline__ void stage_compute(float2 *v, int j0, const float2 *tw) {
  constexpr int R = PL::R[S];
  constexpr int NS = PL::ns(S);
  constexpr int NB = PL::nb(S);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if constexpr (NS > 1) {
      const int j = j0 + b * PL::T;
      const float2 *tk = tw + TwLayout<PL>::off(S) + (j % NS) * (R - 1);
      float2 w[R - 1];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        w[r - 1] = tk[r - 1];
        if (DIR > 0) w[r - 1].y = -w[r - 1].y;
      }
      dft_tw<R, DIR>(v + b * R, w);
    } else {
      dft<R, DIR>(v + b * R);
    }
  }
}

// Synchronisation of a transform group's LDS hand-over.  WAVE: the group lies
// inside one wavefront, whose LDS instructions execute in program order, so a
// compiler-level fence at wavefront scope suffices; otherwise a block barrier.
template <bool WAVE> __device__ __forceinline__ void group_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// hand stage S's outputs to stage S+1's inputs through the group's LDS buffer;
// element i of the group lives at buf[lpad(i) * LS] (LS > 1 interleaves the
// groups of a wave, which keeps their lanes on distinct banks)
template <class PL, int S, bool WAVE, int LS>
__device__ __forceinline__ void stage_exchange(float2 *v, float2 *buf, int j0) {
  constexpr int R = PL::R[S];
  constexpr int NS = PL::ns(S);
  constexpr int B = PL::N / R;
  constexpr int NB = PL::nb(S);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = j0 + b * PL::T;
    if ((NB * PL::T == B) || j < B) {
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lpad(base + r * NS) * LS] = v[b * R + r];
    }
  }
  group_sync<WAVE>();
  constexpr int R2 = PL::R[S + 1];
  constexpr int B2 = PL::N / R2;
  constexpr int NB2 = PL::nb(S + 1);
#pragma unroll
  for (int b = 0; b < NB2; ++b) {
    const int j = j0 + b * PL::T;
    if ((NB2 * PL::T == B2) || j < B2) {
#pragma unroll
      for (int r = 0; r < R2; ++r) v[b * R2 + r] = buf[lpad(j + r * B2) * LS];
    }
  }
  group_sync<WAVE>();
}

// tw: the plan's twiddle table (TwLayout<PL>), in LDS
template <class PL, int DIR, int LS = 1, bool WAVE = true, int S = 0>
__device__ __forceinline__ void fft_run(float2 *v, float2 *buf, int j0, const float2 *tw) {
  stage_compute<PL, S, DIR>(v, j0, tw);
  if constexpr (S + 1 < PL::NST) {
    stage_exchange<PL, S, WAVE, LS>(v, buf, j0);
    fft_run<PL, DIR, LS, WAVE, S + 1>(v, buf, j0, tw);
  }
}

}  // namespace pf
