// C-ABI of the pfista library: plans, validation, dispatch and the solver loop.
// Every numerical step runs in the kernels of pfista_kernels.hpp.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pfista.h"
#include "pfista_kernels.hpp"

struct pfista_plan {
  pfista_desc d;
  int device;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define PF_HIP(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(PFISTA_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define PF_TRY(expr)            \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != PFISTA_OK) return rc_; \
  } while (0)

int launch_status(const char *where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PFISTA_EHIP, "%s: kernel launch failed: %s", where, hipGetErrorString(e));
  return PFISTA_OK;
}

constexpr int kSupportedN[] = {64, 128, 160, 192, 256, 320, 384, 512};
constexpr int kMaxDegree = 8;
constexpr int kNormBlocks = 1024;

bool supported_n(int n) {
  for (int v : kSupportedN)
    if (v == n) return true;
  return false;
}


std::mutex g_tw_mu;
std::vector<int> g_tw_done;

// exp(-2 pi i r k / (Ns R)) for every stage of plan PL, in its TwLayout order
template <class PL> void fill_plan_tw(std::vector<float2> &h, int base) {
  for (int st = 0; st < PL::NST; ++st) {
    const int ns = PL::ns(st), R = PL::R[st];
    if (ns <= 1) continue;
    const int off = base + pf::TwLayout<PL>::off(st);
    for (int k = 0; k < ns; ++k)
      for (int r = 1; r < R; ++r) {
        const double a = -2.0 * M_PI * (double)(r * k) / (double)(ns * R);
        h[off + k * (R - 1) + r - 1] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
  }
}

template <int N> void fill_n(std::vector<float2> &h) {
  const int b = pf::TwBase<N>::v;
  fill_plan_tw<typename pf::Plans<N>::F>(h, b + pf::TwBlock<N>::f);
  fill_plan_tw<typename pf::Plans<N>::I>(h, b + pf::TwBlock<N>::i);
  fill_plan_tw<typename pf::Plans1D<N>::F>(h, b + pf::TwBlock<N>::f1);
  fill_plan_tw<typename pf::Plans1D<N>::I>(h, b + pf::TwBlock<N>::i1);
}

int ensure_twiddles() {
  int dev = 0;
  PF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tw_mu);
  if ((int)g_tw_done.size() <= dev) g_tw_done.resize(dev + 1, 0);
  if (g_tw_done[dev]) return PFISTA_OK;
  std::vector<float2> h(pf::kTwTotal, make_float2(0.f, 0.f));
  fill_n<64>(h);
  fill_n<128>(h);
  fill_n<160>(h);
  fill_n<192>(h);
  fill_n<256>(h);
  fill_n<320>(h);
  fill_n<384>(h);
  fill_n<512>(h);
  PF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(pf::g_tw), h.data(), h.size() * sizeof(float2), 0,
                           hipMemcpyHostToDevice));
  g_tw_done[dev] = 1;
  return PFISTA_OK;
}

// ------------------------------------------------------------------ workspace
struct DevState {
  int k;
  int pad;
  double red[3];
  double data[1];
  double misc[4];
};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t t, img[5], partials, state, rand, total;
  size_t n_img, n_coil, n_partials;
};

Layout layout(const pfista_desc &d) {
  Layout L{};
  const size_t N = d.n, S = d.slices, C = d.coils;
  L.n_img = S * N * N;
  L.n_coil = S * C * N * N;
  const size_t step_blocks = (N / 16) * (N / 16) * S;
  const size_t col_blocks = (N / 16) * S * C;
  L.n_partials = std::max<size_t>({3 * step_blocks, col_blocks, (size_t)kNormBlocks, 16});
  size_t off = 0;
  L.t = off;
  off = align_up(off + L.n_coil * sizeof(float2));
  for (int i = 0; i < 5; ++i) {
    L.img[i] = off;
    off = align_up(off + L.n_img * sizeof(float2));
  }
  L.partials = off;
  off = align_up(off + L.n_partials * sizeof(double));
  L.state = off;
  off = align_up(off + sizeof(DevState));
  L.rand = L.img[4];
  L.total = off;
  return L;
}

template <class T> T *at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

// ------------------------------------------------------------------ validation
int check_plan(const pfista_plan *p) {
  if (!p) return fail(PFISTA_EINVAL, "plan is NULL");
  return PFISTA_OK;
}

int check_ptr(const void *ptr, const char *name, size_t align = 8) {
  if (!ptr) return fail(PFISTA_EINVAL, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(ptr) % align) return fail(PFISTA_EINVAL, "%s is not %zu-byte aligned", name, align);
  return PFISTA_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + nb && pb < pa + na;
}

int check_ops(const pfista_plan *p, const void *sens, const void *mask, const void *ws) {
  PF_TRY(check_plan(p));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(sens, "sens"));
  PF_TRY(check_ptr(mask, "mask", 1));
  PF_TRY(check_ptr(ws, "ws", 16));
  return PFISTA_OK;
}

unsigned blocks_for(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)std::max<size_t>(1, std::min<size_t>(b, 65535));
}

// ------------------------------------------------------------------ per-N dispatch
template <int N> struct Ops {
  using Gm = pf::Geo<N>;

  static void row_fwd(const pfista_desc &d, const float2 *x, const float2 *sens, float2 *t, hipStream_t st,
                      int *k_inc = nullptr) {
    const int tasks = d.slices * N * d.coils;
    const int grid = (tasks + Gm::G - 1) / Gm::G;
    pf::k_row_fwd<N><<<grid, Gm::THREADS, 0, st>>>(x, sens, t, d.coils, tasks, k_inc);
  }

  template <int MODE>
  static void col(const pfista_desc &d, float2 *t, const float2 *kin, float2 *kout, const uint8_t *mask,
                  float a, float b, double *partials, hipStream_t st) {
    const dim3 grid(N / Gm::COLS, d.slices * d.coils);
    if (d.mask_kind == PFISTA_MASK_1D)
      pf::k_col<N, MODE, 1><<<grid, Gm::THREADS, 0, st>>>(t, kin, kout, mask, d.coils, a, b, partials);
    else
      pf::k_col<N, MODE, 0><<<grid, Gm::THREADS, 0, st>>>(t, kin, kout, mask, d.coils, a, b, partials);
  }

  static void row_inv(const pfista_desc &d, const float2 *t, const float2 *sens, float2 *y, const float2 *w,
                      float alpha, float beta, hipStream_t st) {
    int rpw = 1;
    while (rpw * 2 * d.coils <= Gm::G) rpw *= 2;
    const int rows = d.slices * N;
    const int grid = (rows + rpw - 1) / rpw;
    pf::k_row_inv<N><<<grid, Gm::THREADS, 0, st>>>(t, sens, y, w, alpha, beta, d.coils, rows, rpw);
  }

  static void row_inv_fwd(const pfista_desc &d, float2 *t, const float2 *sens, float2 *y, const float2 *w,
                          float alpha, float beta, hipStream_t st) {
    int rpw = 1;
    while (rpw * 2 * d.coils <= Gm::G) rpw *= 2;
    const int rows = d.slices * N;
    const int grid = (rows + rpw - 1) / rpw;
    pf::k_row_inv_fwd<N><<<grid, Gm::THREADS, 0, st>>>(t, sens, y, w, alpha, beta, d.coils, rows, rpw);
  }

  // A chain of m normal applies in which apply k+1's input is apply k's output:
  //   y_k = alpha_k A^H A y_{k-1} + beta_k w_k,  y_0 = x.
  // For a 2-D mask the row passes between applies are fused (2m + 1 kernels).
  static void chain(const pfista_desc &d, const float2 *sens, const uint8_t *mask, const float2 *x, int m,
                    const float *alpha, const float *beta, const float2 *const *w, float2 *const *y, float2 *t,
                    hipStream_t st, int *k_inc) {
    if (d.mask_kind == PFISTA_MASK_1D) {
      const float2 *src = x;
      for (int k = 0; k < m; ++k) {
        normal(d, sens, mask, src, y[k], alpha[k], w[k], beta[k], t, st, k == 0 ? k_inc : nullptr);
        src = y[k];
      }
      return;
    }
    const float inv_n2 = (float)(1.0 / ((double)N * N));
    row_fwd(d, x, sens, t, st, k_inc);
    for (int k = 0; k < m; ++k) {
      col<pf::COL_NORMAL>(d, t, nullptr, nullptr, mask, 1.f, 0.f, nullptr, st);
      if (k + 1 < m)
        row_inv_fwd(d, t, sens, y[k], w[k], alpha[k] * inv_n2, beta[k], st);
      else
        row_inv(d, t, sens, y[k], w[k], alpha[k] * inv_n2, beta[k], st);
    }
  }

  static void normal(const pfista_desc &d, const float2 *sens, const uint8_t *mask, const float2 *x, float2 *y,
                     float alpha, const float2 *w, float beta, float2 *t, hipStream_t st, int *k_inc = nullptr) {
    if (d.mask_kind == PFISTA_MASK_1D) {
      using G1 = pf::Geo1D<N>;
      const dim3 grid(N / G1::COLS, d.slices);
      pf::k_normal_1d<N><<<grid, G1::THREADS, 0, st>>>(x, sens, mask, y, w, alpha / (float)N, beta, d.coils, k_inc);
      return;
    }
    row_fwd(d, x, sens, t, st, k_inc);
    col<pf::COL_NORMAL>(d, t, nullptr, nullptr, mask, 1.f, 0.f, nullptr, st);
    row_inv(d, t, sens, y, w, (float)((double)alpha / ((double)N * N)), beta, st);
  }

  // number of FP64 partial sums the residual column pass writes
  static int resid_blocks(const pfista_desc &d) { return (N / Gm::COLS) * d.slices * d.coils; }

  // kernel passes timed by pfista_profile_normal: the three passes of one apply
  // and the fused inverse+forward row pass of the Horner chain (2-D mask), or
  // the single phase-encode pass; `pass` launches pass k alone
  static int passes(const pfista_desc &d) { return d.mask_kind == PFISTA_MASK_1D ? 1 : 4; }
  static void pass(int k, const pfista_desc &d, const float2 *sens, const uint8_t *mask, const float2 *x, float2 *y,
                   float alpha, const float2 *w, float beta, float2 *t, hipStream_t st) {
    if (d.mask_kind == PFISTA_MASK_1D) {
      normal(d, sens, mask, x, y, alpha, w, beta, t, st);
    } else if (k == 0) {
      row_fwd(d, x, sens, t, st);
    } else if (k == 1) {
      col<pf::COL_NORMAL>(d, t, nullptr, nullptr, mask, 1.f, 0.f, nullptr, st);
    } else if (k == 2) {
      row_inv(d, t, sens, y, w, (float)((double)alpha / ((double)N * N)), beta, st);
    } else {
      row_inv_fwd(d, t, sens, y, w, (float)((double)alpha / ((double)N * N)), beta, st);
    }
  }

  static void forward(const pfista_desc &d, const float2 *sens, const uint8_t *mask, const float2 *x,
                      float2 *kout, float2 *t, hipStream_t st) {
    row_fwd(d, x, sens, t, st);
    col<pf::COL_FWD_OUT>(d, t, nullptr, kout, mask, (float)(1.0 / N), 0.f, nullptr, st);
  }

  static void adjoint(const pfista_desc &d, const float2 *sens, const uint8_t *mask, const float2 *kin,
                      float2 *y, float alpha, float2 *t, hipStream_t st) {
    col<pf::COL_ADJ_IN>(d, t, kin, nullptr, mask, 1.f, 0.f, nullptr, st);
    row_inv(d, t, sens, y, nullptr, (float)((double)alpha / N), 0.f, st);
  }

  // partial sums of |a M F S x - b_scale b|^2, (N/16)*S*C of them
  static void resid(const pfista_desc &d, const float2 *sens, const uint8_t *mask, const float2 *x,
                    const float2 *b, double a, double b_scale, float2 *t, double *partials, hipStream_t st) {
    row_fwd(d, x, sens, t, st);
    col<pf::COL_RESID>(d, t, b, nullptr, mask, (float)(a / N), (float)b_scale, partials, st);
  }

  // k_dev: a valid device int; use_k != 0 takes beta = k / (k + 3) from it
  static void step(const pfista_desc &d, const float2 *z, const float2 *pg, const float2 *xo, float2 *xn,
                   float2 *zn, float pg_scale, float lam, float beta, const int *k_dev, int use_k,
                   double *partials, hipStream_t st) {
    const dim3 grid(N / 16, N / 16, d.slices);
    switch (d.haar_levels) {
      case 1: pf::k_step<1><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials); break;
      case 2: pf::k_step<2><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials); break;
      case 3: pf::k_step<3><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials); break;
      default: pf::k_step<4><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials); break;
    }
  }
};

// dispatch helper: calls F<N>::run(args...) for the plan's N
#define PF_DISPATCH(n, CALL)                   \
  switch (n) {                                 \
    case 64: { constexpr int NN = 64; CALL; } break;   \
    case 128: { constexpr int NN = 128; CALL; } break; \
    case 160: { constexpr int NN = 160; CALL; } break; \
    case 192: { constexpr int NN = 192; CALL; } break; \
    case 256: { constexpr int NN = 256; CALL; } break; \
    case 320: { constexpr int NN = 320; CALL; } break; \
    case 384: { constexpr int NN = 384; CALL; } break; \
    case 512: { constexpr int NN = 512; CALL; } break; \
    default: break;                            \
  }

const float2 *F2(const pfista_c32 *p) { return reinterpret_cast<const float2 *>(p); }
float2 *F2(pfista_c32 *p) { return reinterpret_cast<float2 *>(p); }

void normal_op(const pfista_desc &d, const pfista_c32 *sens, const uint8_t *mask, const float2 *x, float2 *y,
               float alpha, const float2 *w, float beta, void *ws, hipStream_t st, int *k_inc = nullptr) {
  const Layout L = layout(d);
  float2 *t = at<float2>(ws, L.t);
  PF_DISPATCH(d.n, Ops<NN>::normal(d, F2(sens), mask, x, y, alpha, w, beta, t, st, k_inc));
}

void reduce(const double *partials, int count, int width, double *out, int *k_dev, hipStream_t st) {
  pf::k_reduce<<<1, 64, 0, st>>>(partials, count, width, out, k_dev);
}

void norm2_dev(const float2 *v, size_t n, double *partials, double *out, hipStream_t st) {
  const unsigned nb = (unsigned)std::min<size_t>(kNormBlocks, std::max<size_t>(1, (n + 255) / 256));
  pf::k_norm2<<<nb, 256, 0, st>>>(v, n, partials);
  reduce(partials, (int)nb, 1, out, nullptr, st);
}

// Horner recursion of the nested form c0 I + N'(c1 I + N'(... c_d I)):
// h = c_d g; h = c_i g + N' h for i = d-1 .. 0.  The first apply folds c_d
// into its alpha; optionally preceded by the gradient apply g = N' z - A'^H b'
// (then `pre_x` = z, `pre_w` = A'^H b', output in g), all as one chain.
void grad_poly_op(const pfista_desc &d, const pfista_c32 *sens, const uint8_t *mask, double inv_l,
                  const std::vector<double> &c, const float2 *pre_x, const float2 *pre_w, float2 *g,
                  float2 *out, void *ws, hipStream_t st, int *k_inc) {
  const int deg = (int)c.size() - 1;
  const Layout L = layout(d);
  float2 *t = at<float2>(ws, L.t);
  float alpha[kMaxDegree + 1], beta[kMaxDegree + 1];
  const float2 *w[kMaxDegree + 1];
  float2 *y[kMaxDegree + 1];
  int m = 0;
  if (pre_x) {
    alpha[m] = (float)inv_l; beta[m] = -1.f; w[m] = pre_w; y[m] = g; ++m;
  }
  for (int i = 1; i <= deg; ++i) {
    alpha[m] = (float)(i == 1 ? c[deg] * inv_l : inv_l);
    beta[m] = (float)c[deg - i];
    w[m] = g;
    y[m] = out;
    ++m;
  }
  if (m > 0) {
    const float2 *x0 = pre_x ? pre_x : g;
    PF_DISPATCH(d.n, Ops<NN>::chain(d, F2(sens), mask, x0, m, alpha, beta, w, y, t, st, k_inc));
  }
  if (deg == 0 && !pre_x) pf::k_scale<<<blocks_for(L.n_img), 256, 0, st>>>(g, out, L.n_img, (float)c[0]);
}

void poly_op(const pfista_desc &d, const pfista_c32 *sens, const uint8_t *mask, double inv_l,
             const std::vector<double> &c, const float2 *g, float2 *out, void *ws, hipStream_t st) {
  grad_poly_op(d, sens, mask, inv_l, c, nullptr, nullptr, const_cast<float2 *>(g), out, ws, st, nullptr);
}

int l2_coefficients(int d, std::vector<double> &c) {
  if (d < 0 || d > kMaxDegree) return fail(PFISTA_UNSUPPORTED, "degree %d outside 0..%d", d, kMaxDegree);
  // c_j = (-1)^j / (d+2)^2 * sum_{k=j+1}^{d+1} (2k+1) C(k, j+1) C(k+j+1, j+1)
  auto binom = [](long long n, long long k) {
    long long r = 1;
    for (long long i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  c.assign(d + 1, 0.0);
  const double den = (double)((d + 2) * (d + 2));
  for (int j = 0; j <= d; ++j) {
    long long s = 0;
    for (int k = j + 1; k <= d + 1; ++k) s += (long long)(2 * k + 1) * binom(k, j + 1) * binom(k + j + 1, j + 1);
    c[j] = ((j % 2) ? -(double)s : (double)s) / den;
  }
  return PFISTA_OK;
}

// Weighted L2 design (w(z) = z^alpha): normal equations sum_j c_j m_(i+j+2) =
// m_(i+1), m_k = 1/(alpha + k + 1), by Gaussian elimination with partial
// pivoting in long double.
int weighted_coefficients(int d, double alpha, std::vector<double> &c) {
  if (d < 0 || d > kMaxDegree) return fail(PFISTA_UNSUPPORTED, "degree %d outside 0..%d", d, kMaxDegree);
  if (!(alpha > -1.0) || !std::isfinite(alpha)) return fail(PFISTA_EINVAL, "alpha must be finite and > -1");
  const int n = d + 1;
  std::vector<long double> a((size_t)n * (n + 1));
  auto m = [&](int k) { return 1.0L / ((long double)alpha + (long double)k + 1.0L); };
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) a[(size_t)i * (n + 1) + j] = m(i + j + 2);
    a[(size_t)i * (n + 1) + n] = m(i + 1);
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * (n + 1) + col]) > std::fabs(a[(size_t)piv * (n + 1) + col])) piv = r;
    if (piv != col)
      for (int k = 0; k <= n; ++k) std::swap(a[(size_t)col * (n + 1) + k], a[(size_t)piv * (n + 1) + k]);
    const long double pv = a[(size_t)col * (n + 1) + col];
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const long double f = a[(size_t)r * (n + 1) + col] / pv;
      for (int k = col; k <= n; ++k) a[(size_t)r * (n + 1) + k] -= f * a[(size_t)col * (n + 1) + k];
    }
  }
  c.resize(n);
  for (int i = 0; i < n; ++i) c[i] = (double)(a[(size_t)i * (n + 1) + n] / a[(size_t)i * (n + 1) + i]);
  return PFISTA_OK;
}

// L-infinity (Chebyshev) design for a known smallest eigenvalue mu in (0, 1):
// r(z) = T_(d+1)(u0 + u1 z) / T_(d+1)(u0), u0 = (1+mu)/(1-mu), u1 = -2/(1-mu),
// expanded in powers of z by T_(n+1) = 2u T_n - T_(n-1) (long double); p = (1 - r)/z.
int chebyshev_coefficients(int d, double mu, std::vector<double> &c) {
  if (d < 0 || d > kMaxDegree) return fail(PFISTA_UNSUPPORTED, "degree %d outside 0..%d", d, kMaxDegree);
  if (!(mu > 0.0 && mu < 1.0)) return fail(PFISTA_EINVAL, "mu must lie in (0, 1)");
  const long double u0 = (1.0L + mu) / (1.0L - mu), u1 = -2.0L / (1.0L - mu);
  std::vector<long double> tp{1.0L}, tc{u0, u1};
  for (int it = 0; it < d; ++it) {
    std::vector<long double> nx(tc.size() + 1, 0.0L);
    for (size_t i = 0; i < tc.size(); ++i) {
      nx[i] += 2.0L * u0 * tc[i];
      nx[i + 1] += 2.0L * u1 * tc[i];
    }
    for (size_t i = 0; i < tp.size(); ++i) nx[i] -= tp[i];
    tp = tc;
    tc = nx;
  }
  c.resize(d + 1);
  for (int j = 0; j <= d; ++j) c[j] = (double)(-tc[j + 1] / tc[0]);
  return PFISTA_OK;
}

}  // namespace

// ============================================================================ C-ABI
extern "C" {

const char *pfista_last_error(void) { return g_err.c_str(); }

int pfista_plan_create(pfista_plan **out, const pfista_desc *d) {
  if (!out || !d) return fail(PFISTA_EINVAL, "out/desc is NULL");
  *out = nullptr;
  if (!supported_n(d->n)) return fail(PFISTA_UNSUPPORTED, "image side %d not in {64,128,160,192,256,320,384,512}", d->n);
  if (d->coils < 1) return fail(PFISTA_EINVAL, "coils must be >= 1 (got %d)", d->coils);
  if (d->slices < 0) return fail(PFISTA_EINVAL, "slices must be >= 0 (got %d)", d->slices);
  if ((long long)d->slices * d->coils > 65535) return fail(PFISTA_UNSUPPORTED, "slices * coils > 65535");
  if (d->haar_levels < 1 || d->haar_levels > 4)
    return fail(PFISTA_UNSUPPORTED, "haar_levels %d outside 1..4", d->haar_levels);
  if (d->mask_kind != PFISTA_MASK_2D && d->mask_kind != PFISTA_MASK_1D)
    return fail(PFISTA_EINVAL, "mask_kind %d", d->mask_kind);
  PF_TRY(ensure_twiddles());
  pfista_plan *p = new (std::nothrow) pfista_plan;
  if (!p) return fail(PFISTA_EINVAL, "out of host memory");
  p->d = *d;
  PF_HIP(hipGetDevice(&p->device));
  *out = p;
  return PFISTA_OK;
}

void pfista_plan_destroy(pfista_plan *p) { delete p; }

size_t pfista_workspace_bytes(const pfista_plan *p) {
  if (!p) return 0;
  return layout(p->d).total;
}

int pfista_poly_coefficients(int degree, double *coef) {
  if (!coef) return fail(PFISTA_EINVAL, "coef is NULL");
  std::vector<double> c;
  PF_TRY(l2_coefficients(degree, c));
  std::copy(c.begin(), c.end(), coef);
  return PFISTA_OK;
}

int pfista_poly_coefficients_weighted(int degree, double alpha, double *coef) {
  if (!coef) return fail(PFISTA_EINVAL, "coef is NULL");
  std::vector<double> c;
  PF_TRY(weighted_coefficients(degree, alpha, c));
  std::copy(c.begin(), c.end(), coef);
  return PFISTA_OK;
}

int pfista_poly_coefficients_chebyshev(int degree, double mu, double *coef) {
  if (!coef) return fail(PFISTA_EINVAL, "coef is NULL");
  std::vector<double> c;
  PF_TRY(chebyshev_coefficients(degree, mu, c));
  std::copy(c.begin(), c.end(), coef);
  return PFISTA_OK;
}

int pfista_normal_apply(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *x,
                        pfista_c32 *y, float alpha, const pfista_c32 *w, float beta, void *ws,
                        hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(x, "x"));
  PF_TRY(check_ptr(y, "y"));
  if (w) PF_TRY(check_ptr(w, "w"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  const size_t nb = L.n_img * sizeof(float2);
  if (overlaps(x, nb, y, nb)) return fail(PFISTA_EINVAL, "y overlaps x");
  if (w && w != y && overlaps(w, nb, y, nb)) return fail(PFISTA_EINVAL, "w partially overlaps y");
  normal_op(p->d, sens, mask, F2(x), F2(y), alpha, w ? F2(w) : nullptr, beta, ws, stream);
  return launch_status("pfista_normal_apply");
}

int pfista_poly_apply(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, double inv_l,
                      const double *coef, int degree, const pfista_c32 *g, pfista_c32 *out, void *ws,
                      hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(g, "g"));
  PF_TRY(check_ptr(out, "out"));
  if (!coef) return fail(PFISTA_EINVAL, "coef is NULL");
  if (degree < 0 || degree > kMaxDegree) return fail(PFISTA_UNSUPPORTED, "degree %d outside 0..%d", degree, kMaxDegree);
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  const size_t nb = L.n_img * sizeof(float2);
  if (overlaps(g, nb, out, nb)) return fail(PFISTA_EINVAL, "out overlaps g");
  std::vector<double> c(coef, coef + degree + 1);
  poly_op(p->d, sens, mask, inv_l, c, F2(g), F2(out), ws, stream);
  return launch_status("pfista_poly_apply");
}

int pfista_step(const pfista_plan *p, const pfista_c32 *z, const pfista_c32 *pg, const pfista_c32 *x_old,
                pfista_c32 *x_new, pfista_c32 *z_new, float lambda, float beta_k, double *red, void *ws,
                hipStream_t stream) {
  PF_TRY(check_plan(p));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(z, "z", 16));
  PF_TRY(check_ptr(pg, "pg", 16));
  PF_TRY(check_ptr(x_old, "x_old", 16));
  PF_TRY(check_ptr(x_new, "x_new", 16));
  PF_TRY(check_ptr(z_new, "z_new", 16));
  PF_TRY(check_ptr(red, "red"));
  PF_TRY(check_ptr(ws, "ws", 16));
  if (!(lambda >= 0.f)) return fail(PFISTA_EINVAL, "lambda must be >= 0");
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  double *partials = at<double>(ws, L.partials);
  DevState *ds = at<DevState>(ws, L.state);
  PF_DISPATCH(p->d.n, Ops<NN>::step(p->d, F2(z), F2(pg), F2(x_old), F2(x_new), F2(z_new), 1.f, lambda, beta_k,
                                    &ds->k, 0, partials, stream));
  const int nblk = (p->d.n / 16) * (p->d.n / 16) * p->d.slices;
  reduce(partials, nblk, 3, red, nullptr, stream);
  return launch_status("pfista_step");
}

int pfista_forward(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *x,
                   pfista_c32 *kspace, void *ws, hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(x, "x"));
  PF_TRY(check_ptr(kspace, "kspace"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  float2 *t = at<float2>(ws, L.t);
  PF_DISPATCH(p->d.n, Ops<NN>::forward(p->d, F2(sens), mask, F2(x), F2(kspace), t, stream));
  return launch_status("pfista_forward");
}

int pfista_adjoint(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *kspace,
                   pfista_c32 *y, float alpha, void *ws, hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(kspace, "kspace"));
  PF_TRY(check_ptr(y, "y"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  float2 *t = at<float2>(ws, L.t);
  PF_DISPATCH(p->d.n, Ops<NN>::adjoint(p->d, F2(sens), mask, F2(kspace), F2(y), alpha, t, stream));
  return launch_status("pfista_adjoint");
}

int pfista_data_term(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *b,
                     const pfista_c32 *x, double inv_l, double b_scale, double *out, void *ws,
                     hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (!out) return fail(PFISTA_EINVAL, "out is NULL");
  if (p->d.slices == 0) {
    *out = 0.0;
    return PFISTA_OK;
  }
  PF_TRY(check_ptr(b, "b"));
  PF_TRY(check_ptr(x, "x"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) {
    *out = 0.0;
    return PFISTA_OK;
  }
  float2 *t = at<float2>(ws, L.t);
  double *partials = at<double>(ws, L.partials);
  DevState *ds = at<DevState>(ws, L.state);
  PF_DISPATCH(p->d.n, Ops<NN>::resid(p->d, F2(sens), mask, F2(x), F2(b), std::sqrt(inv_l), b_scale, t, partials,
                                     stream));
  int cnt = 0;
  PF_DISPATCH(p->d.n, cnt = Ops<NN>::resid_blocks(p->d));
  reduce(partials, cnt, 1, ds->data, nullptr, stream);
  PF_TRY(launch_status("pfista_data_term"));
  double h = 0.0;
  PF_HIP(hipMemcpyAsync(&h, ds->data, sizeof(double), hipMemcpyDeviceToHost, stream));
  PF_HIP(hipStreamSynchronize(stream));
  *out = 0.5 * h;
  return PFISTA_OK;
}

int pfista_power_iteration(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, pfista_c32 *v,
                           int iters, double *lam_max, void *ws, hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (!lam_max) return fail(PFISTA_EINVAL, "lam_max is NULL");
  if (p->d.slices == 0) {
    *lam_max = 0.0;
    return PFISTA_OK;
  }
  if (iters < 1) return fail(PFISTA_EINVAL, "iters must be >= 1");
  const Layout L = layout(p->d);
  if (L.n_img == 0) {
    *lam_max = 0.0;
    return PFISTA_OK;
  }
  if (v) PF_TRY(check_ptr(v, "v"));
  float2 *cur = v ? F2(v) : at<float2>(ws, L.img[4]);
  float2 *nxt = at<float2>(ws, L.img[3]);
  double *partials = at<double>(ws, L.partials);
  DevState *ds = at<DevState>(ws, L.state);
  if (!v) pf::k_random<<<blocks_for(L.n_img), 256, 0, stream>>>(cur, L.n_img, 0ull);
  norm2_dev(cur, L.n_img, partials, ds->misc, stream);
  pf::k_normalise<<<blocks_for(L.n_img), 256, 0, stream>>>(cur, L.n_img, ds->misc);
  for (int it = 0; it < iters; ++it) {
    normal_op(p->d, sens, mask, cur, nxt, 1.f, nullptr, 0.f, ws, stream);
    norm2_dev(nxt, L.n_img, partials, ds->misc, stream);
    pf::k_normalise<<<blocks_for(L.n_img), 256, 0, stream>>>(nxt, L.n_img, ds->misc);
    std::swap(cur, nxt);
  }
  PF_TRY(launch_status("pfista_power_iteration"));
  if (v && cur != F2(v)) PF_HIP(hipMemcpyAsync(v, cur, L.n_img * sizeof(float2), hipMemcpyDeviceToDevice, stream));
  double h = 0.0;
  PF_HIP(hipMemcpyAsync(&h, ds->misc, sizeof(double), hipMemcpyDeviceToHost, stream));
  PF_HIP(hipStreamSynchronize(stream));
  *lam_max = std::sqrt(h);
  return PFISTA_OK;
}

int pfista_profile_normal(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                          const pfista_c32 *x, pfista_c32 *y, int reps, float *pass_ms, int *npasses, void *ws,
                          hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (!pass_ms || !npasses) return fail(PFISTA_EINVAL, "pass_ms/npasses is NULL");
  if (reps < 1) return fail(PFISTA_EINVAL, "reps must be >= 1");
  const pfista_desc &d = p->d;
  int np = 0;
  PF_DISPATCH(d.n, np = Ops<NN>::passes(d));
  *npasses = np;
  for (int k = 0; k < np; ++k) pass_ms[k] = 0.f;
  if (d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(x, "x"));
  PF_TRY(check_ptr(y, "y"));
  const Layout L = layout(d);
  const size_t nb = L.n_img * sizeof(float2);
  if (overlaps(x, nb, y, nb)) return fail(PFISTA_EINVAL, "y overlaps x");
  float2 *t = at<float2>(ws, L.t);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PF_HIP(hipEventCreate(&e0));
  PF_HIP(hipEventCreate(&e1));
  int rc = PFISTA_OK;
  // each pass `reps` times back to back (every pass leaves valid inputs for the
  // next: the column pass is a projection, the row passes recompute their outputs)
  for (int k = 0; k < np && rc == PFISTA_OK; ++k) {
    hipError_t he = hipEventRecord(e0, stream);
    for (int r = 0; r < reps && he == hipSuccess; ++r)
      PF_DISPATCH(d.n, Ops<NN>::pass(k, d, F2(sens), mask, F2(x), F2(y), 1.f, nullptr, 0.f, t, stream));
    if (he == hipSuccess) he = hipEventRecord(e1, stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) {
      rc = fail(PFISTA_EHIP, "pfista_profile_normal: %s", hipGetErrorString(he));
      break;
    }
    rc = launch_status("pfista_profile_normal");
    pass_ms[k] = ms / (float)reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int pfista_solve(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *b,
                 const pfista_params *prm, pfista_c32 *x_io, pfista_c32 *z_io, double *history,
                 pfista_report *rep, void *ws, hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.slices == 0) {
    if (rep) {
      *rep = pfista_report{};
      rep->objective = NAN;
    }
    return PFISTA_OK;
  }
  PF_TRY(check_ptr(b, "b"));
  PF_TRY(check_ptr(x_io, "x_io", 16));
  if (z_io) PF_TRY(check_ptr(z_io, "z_io", 16));
  if (!prm) return fail(PFISTA_EINVAL, "params is NULL");
  if (prm->max_iter < 0) return fail(PFISTA_EINVAL, "max_iter < 0");
  if (prm->check_every < 1 || prm->check_every > 4096) return fail(PFISTA_EINVAL, "check_every outside 1..4096");
  if (!(prm->lambda >= 0.0)) return fail(PFISTA_EINVAL, "lambda must be >= 0");
  if (prm->k0 < 0 || (prm->k0 > 0 && !z_io)) return fail(PFISTA_EINVAL, "resume (k0 > 0) needs z_io");
  if (prm->inv_l < 0.0) return fail(PFISTA_EINVAL, "inv_l < 0");
  if (prm->inv_l == 0.0 && prm->power_iters < 1) return fail(PFISTA_EINVAL, "inv_l == 0 needs power_iters >= 1");
  std::vector<double> c;
  if (prm->coef) {
    if (prm->degree < 0 || prm->degree > kMaxDegree) return fail(PFISTA_UNSUPPORTED, "degree %d", prm->degree);
    c.assign(prm->coef, prm->coef + prm->degree + 1);
  } else {
    PF_TRY(l2_coefficients(prm->degree, c));
  }
  const pfista_desc &d = p->d;
  const Layout L = layout(d);
  pfista_report r{};
  r.objective = NAN;
  r.status = PFISTA_OK;
  if (L.n_img == 0) {
    if (rep) *rep = r;
    return PFISTA_OK;
  }
  float2 *ahb = at<float2>(ws, L.img[0]);
  float2 *g = at<float2>(ws, L.img[1]);
  float2 *pgb = at<float2>(ws, L.img[2]);
  float2 *zb = z_io ? F2(z_io) : at<float2>(ws, L.img[4]);
  float2 *x = F2(x_io);
  double *partials = at<double>(ws, L.partials);
  DevState *ds = at<DevState>(ws, L.state);
  const size_t nbytes = L.n_img * sizeof(float2);
  if (overlaps(x, nbytes, zb, nbytes)) return fail(PFISTA_EINVAL, "x_io overlaps z_io");

  // ---- setup: ||b||, L, A'^H b'
  double h[4] = {0, 0, 0, 0};
  norm2_dev(F2(b), L.n_coil, partials, ds->misc, stream);
  PF_TRY(launch_status("pfista_solve(norm)"));
  PF_HIP(hipMemcpyAsync(h, ds->misc, sizeof(double), hipMemcpyDeviceToHost, stream));
  PF_HIP(hipStreamSynchronize(stream));
  const double bnorm = std::sqrt(h[0]);
  r.bnorm = bnorm;
  double inv_l = prm->inv_l;
  if (inv_l == 0.0) {
    double lam = 0.0;
    PF_TRY(pfista_power_iteration(p, sens, mask, nullptr, prm->power_iters, &lam, ws, stream));
    if (!(lam > 0.0)) return fail(PFISTA_EINVAL, "power iteration gave %g", lam);
    inv_l = 1.0 / (1.01 * lam);
  }
  r.inv_l = inv_l;
  if (!(bnorm > 0.0)) {
    pf::k_fill<<<blocks_for(L.n_img), 256, 0, stream>>>(x, L.n_img, make_float2(0.f, 0.f));
    PF_TRY(launch_status("pfista_solve(zero)"));
    r.objective = 0.0;
    if (rep) *rep = r;
    return PFISTA_OK;
  }
  PF_DISPATCH(d.n, Ops<NN>::adjoint(d, F2(sens), mask, F2(b), ahb, (float)(std::sqrt(inv_l) / bnorm),
                                    at<float2>(ws, L.t), stream));
  if (prm->k0 == 0) {
    pf::k_fill<<<blocks_for(L.n_img), 256, 0, stream>>>(x, L.n_img, make_float2(0.f, 0.f));
    pf::k_fill<<<blocks_for(L.n_img), 256, 0, stream>>>(zb, L.n_img, make_float2(0.f, 0.f));
  }
  const int k0 = prm->k0;
  const int k_start = k0 - 1;   // the first gradient apply advances it to k0
  PF_HIP(hipMemcpyAsync(&ds->k, &k_start, sizeof(int), hipMemcpyHostToDevice, stream));
  PF_TRY(launch_status("pfista_solve(setup)"));

  const int deg = (int)c.size() - 1;
  const float lam = (float)prm->lambda;
  const int nstep = (d.n / 16) * (d.n / 16) * d.slices;
  auto body = [&]() {
    // g = N' z - A'^H b' then pg = p(N') g as one chain of d + 1 applies (its
    // first kernel advances the iteration counter k); then the fused step
    grad_poly_op(d, sens, mask, inv_l, c, zb, ahb, g, pgb, ws, stream, &ds->k);
    const float2 *pg = deg == 0 ? g : pgb;
    const float pg_scale = deg == 0 ? (float)c[0] : 1.f;
    // momentum off (Algorithms 1 and 3): beta = 0, so z_(k+1) = x_(k+1)
    const int use_k = prm->momentum ? 1 : 0;
    PF_DISPATCH(d.n, Ops<NN>::step(d, zb, pg, x, x, zb, pg_scale, lam, 0.f, &ds->k, use_k, partials, stream));
  };

  hipGraphExec_t gexec = nullptr;
  int gunroll = 0;
  if (prm->graph_iters > 0 && stream != nullptr) {
    gunroll = std::min(prm->graph_iters, prm->check_every);
    hipGraph_t graph = nullptr;
    PF_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < gunroll; ++i) body();
    hipError_t ce = hipStreamEndCapture(stream, &graph);
    if (ce != hipSuccess) return fail(PFISTA_EHIP, "graph capture: %s", hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(PFISTA_EHIP, "graph instantiate: %s", hipGetErrorString(ie));
  }

  int done = 0, nchecks = 0;
  int status = PFISTA_OK;
  while (done < prm->max_iter) {
    const int chunk = std::min(prm->check_every, prm->max_iter - done);
    int left = chunk;
    if (gexec) {
      while (left >= gunroll) {
        hipError_t le = hipGraphLaunch(gexec, stream);
        if (le != hipSuccess) {
          (void)hipGraphExecDestroy(gexec);
          return fail(PFISTA_EHIP, "graph launch: %s", hipGetErrorString(le));
        }
        left -= gunroll;
      }
    }
    for (; left > 0; --left) body();
    done += chunk;
    // FP64 sums of the last step of the chunk (its partials are still in place)
    reduce(partials, nstep, 3, ds->red, nullptr, stream);
    int lrc = launch_status("pfista_solve(loop)");
    if (lrc != PFISTA_OK) {
      if (gexec) (void)hipGraphExecDestroy(gexec);
      return lrc;
    }
    double F = NAN;
    if (prm->eval_objective) {
      PF_DISPATCH(d.n, Ops<NN>::resid(d, F2(sens), mask, x, F2(b), std::sqrt(inv_l), 1.0 / bnorm,
                                      at<float2>(ws, L.t), partials, stream));
      int cnt = 0;
      PF_DISPATCH(d.n, cnt = Ops<NN>::resid_blocks(d));
      reduce(partials, cnt, 1, ds->data, nullptr, stream);
    }
    hipError_t me = hipMemcpyAsync(h, ds->red, 4 * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (me == hipSuccess) me = hipStreamSynchronize(stream);
    if (me != hipSuccess) {
      if (gexec) (void)hipGraphExecDestroy(gexec);
      return fail(PFISTA_EHIP, "pfista_solve(check): %s", hipGetErrorString(me));
    }
    const double l1 = h[0], dx2 = h[1], xn2 = h[2];
    r.l1 = l1;
    r.rel_change = xn2 > 0 ? std::sqrt(dx2 / xn2) : 0.0;
    if (prm->eval_objective) {
      F = 0.5 * h[3] + prm->lambda * l1;
      r.objective = F;
      if (history) history[nchecks] = F;
    }
    ++nchecks;
    const bool bad = !std::isfinite(l1) || !std::isfinite(dx2) || !std::isfinite(xn2) ||
                     (prm->eval_objective && (!std::isfinite(F) || F > 5.0));
    if (bad) {
      status = PFISTA_DIVERGED;
      fail(PFISTA_DIVERGED, "diverged after %d iterations (objective %g)", k0 + done, F);
      break;
    }
    if (prm->tol > 0 && r.rel_change <= prm->tol) break;
    if (prm->f_stop > 0 && prm->eval_objective && F <= prm->f_stop) break;
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  r.iters = done;
  r.status = status;
  r.normal_applies = (long long)done * (deg + 1);
  if (rep) *rep = r;
  return status;
}

}  // extern "C"
