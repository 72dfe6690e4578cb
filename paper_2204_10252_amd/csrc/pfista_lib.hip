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

// the Toeplitz operator runs transforms of length 2n
bool supported_toeplitz_n(int n) { return n <= 256 && supported_n(2 * n); }


std::mutex g_tw_mu;
std::vector<int> g_tw_done;

// Static transform buffer of pfista_normal_apply_noalloc, one per device.  Host
// code never uses the array's name as an address: each device's copy is looked
// up once (hipGetSymbolAddress, with that device current) when the first plan
// on the device is created, and that pointer is what kernels receive.
__device__ __align__(256) unsigned char scratch[PFISTA_STATIC_SCRATCH_BYTES];
std::vector<void *> g_scratch_ptr;

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
  fill_plan_tw<typename pf::PlansV<N, 1>::F>(h, b + pf::TwBlock<N>::fa);
  fill_plan_tw<typename pf::PlansV<N, 1>::I>(h, b + pf::TwBlock<N>::ia);
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
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  void *sp = nullptr;
  PF_HIP(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
  if (!sp) return fail(PFISTA_EHIP, "no device address for the static scratch array");
  g_scratch_ptr[dev] = sp;
  g_tw_done[dev] = 1;
  return PFISTA_OK;
}

// this device's static scratch array (set up with its first plan), or null
void *device_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_tw_mu);
  return dev >= 0 && dev < (int)g_scratch_ptr.size() ? g_scratch_ptr[dev] : nullptr;
}

// ------------------------------------------------------------------ workspace
struct DevState {
  int k;
  int pad;
  double red[3];
  double data[1];
  double misc[4];
};

// the solver's iteration counter, set on the stream by a kernel (no host
// memory is read after the call returns); the next chain advances it by one
void set_counter(DevState *ds, int k, hipStream_t st) { pf::k_set_counter<<<1, 64, 0, st>>>(&ds->k, k); }

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
  // the Toeplitz operator's transform buffer holds N rows of length 2N per coil image
  const size_t n_t = d.mask_kind == PFISTA_TOEPLITZ ? 2 * L.n_coil : L.n_coil;
  const size_t step_blocks = (N / 16) * (N / 16) * S;
  const size_t col_blocks = (N / 16) * S * C;
  L.n_partials = std::max<size_t>({3 * step_blocks, col_blocks, (size_t)kNormBlocks, 16});
  size_t off = 0;
  L.t = off;
  off = align_up(off + n_t * sizeof(float2));
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

// pfista_solve's workspace: the layout above, then (phase-encode plans) the
// packed coil maps its loop reads when it runs at least kPackMinApplies applies
constexpr long long kPackMinApplies = 12;
size_t solve_packed_off(const pfista_desc &d) { return align_up(layout(d).total); }
size_t solve_ws_bytes(const pfista_desc &d) {
  const Layout L = layout(d);
  return d.mask_kind == PFISTA_MASK_1D ? solve_packed_off(d) + align_up(L.n_coil * sizeof(float2)) : L.total;
}

// ------------------------------------------------------------------ validation
// a plan (or batch) belongs to the device that was current when it was created
int check_device(int dev) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(PFISTA_EHIP, "hipGetDevice failed");
  if (cur != dev) return fail(PFISTA_EINVAL, "created on device %d, but device %d is current", dev, cur);
  return PFISTA_OK;
}

int check_plan(const pfista_plan *p) {
  if (!p) return fail(PFISTA_EINVAL, "plan is NULL");
  return check_device(p->device);
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
// What a launch needs to know about the slices it covers.  A plan's slices all
// have `coils` coils (cb = cs = nullptr); a batch group's slices may differ, and
// then cb (device, slices + 1 entries) holds the first coil image of every
// slice and cs (device, one entry per coil image) the slice of every image.
struct Shape {
  int slices;
  int coils;        // coil count when uniform
  int images;       // coil images in all
  int haar_levels;
  int mask_kind;
  const int *cb;
  const int *cs;
  int cmin;         // smallest coil count of a slice (sizes the coil-combine passes)
  int rpw_mult;     // rows per coil-combine block, as a multiple of the default
  int fused;        // fuse the row passes between the applies of a chain
  int packed;       // phase-encode mask: `sens` holds the packed coil maps
};

Shape shape_of(const pfista_desc &d) {
  return Shape{d.slices, d.coils, d.slices * d.coils, d.haar_levels, d.mask_kind, nullptr, nullptr, d.coils, 1, 1, 0};
}

// Toeplitz normal operator with transforms of length M = 2N (image side N);
// `kern` is the real M x M kernel per slice.
template <int M> struct ToeOps {
  using Gm = pf::Geo<M>;
  static constexpr int N = M / 2;

  static int rows_per_block(const Shape &d) {
    int rpw = 1;
    while (rpw * 2 * d.cmin <= Gm::G) rpw *= 2;
    return rpw;
  }
  static void row_fwd(const Shape &d, const float2 *x, const float2 *sens, float2 *t, hipStream_t st, int *k_inc) {
    const int tasks = d.slices * N * d.coils;
    pf::k_trow_fwd<M><<<(tasks + Gm::G - 1) / Gm::G, Gm::THREADS, 0, st>>>(x, sens, t, d.coils, tasks, k_inc);
  }
  static void col(const Shape &d, float2 *t, const float *kern, hipStream_t st) {
    pf::k_tcol<M><<<dim3(M / Gm::COLS, d.slices * d.coils), Gm::THREADS, 0, st>>>(t, kern, d.coils);
  }
  static void row_inv(const Shape &d, const float2 *t, const float2 *sens, float2 *y, const float2 *w, float alpha,
                      float beta, hipStream_t st) {
    const int rpw = rows_per_block(d);
    const int rows = d.slices * N;
    pf::k_trow_inv<M><<<(rows + rpw - 1) / rpw, Gm::THREADS, 0, st>>>(
        t, sens, y, w, (float)((double)alpha / ((double)M * M)), beta, d.coils, rows, rpw);
  }
  static void normal(const Shape &d, const float2 *sens, const float *kern, const float2 *x, float2 *y, float alpha,
                     const float2 *w, float beta, float2 *t, hipStream_t st, int *k_inc) {
    row_fwd(d, x, sens, t, st, k_inc);
    col(d, t, kern, st);
    row_inv(d, t, sens, y, w, alpha, beta, st);
  }
  static void pass(int k, const Shape &d, const float2 *sens, const float *kern, const float2 *x, float2 *y,
                   float alpha, const float2 *w, float beta, float2 *t, hipStream_t st) {
    if (k == 0) row_fwd(d, x, sens, t, st, nullptr);
    else if (k == 1) col(d, t, kern, st);
    else row_inv(d, t, sens, y, w, alpha, beta, st);
  }
};

template <int N, int V = 0> struct Ops {
  using Gm = pf::Geo<N, V>;

  static void row_fwd(const Shape &d, const float2 *x, const float2 *sens, float2 *t, hipStream_t st,
                      int *k_inc = nullptr) {
    const int tasks = d.images * N;
    const int grid = (tasks + Gm::G - 1) / Gm::G;
    if (d.cb) pf::k_row_fwd<N, V, true><<<grid, Gm::THREADS, 0, st>>>(x, sens, t, d.coils, tasks, k_inc, d.cb, d.slices);
    else pf::k_row_fwd<N, V, false><<<grid, Gm::THREADS, 0, st>>>(x, sens, t, d.coils, tasks, k_inc, nullptr, d.slices);
  }

  template <int MODE>
  static void col(const Shape &d, float2 *t, const float2 *kin, float2 *kout, const uint8_t *mask,
                  float a, float b, double *partials, hipStream_t st) {
    const dim3 grid(N / Gm::COLS, d.images);
    if constexpr (V == 0) {
      if (d.mask_kind == PFISTA_MASK_1D) {
        pf::k_col<N, MODE, 1, V><<<grid, Gm::THREADS, 0, st>>>(t, kin, kout, mask, d.coils, a, b, partials, d.cs);
        return;
      }
    }
    pf::k_col<N, MODE, 0, V><<<grid, Gm::THREADS, 0, st>>>(t, kin, kout, mask, d.coils, a, b, partials, d.cs);
  }

  // rows per block of the coil-combine passes: by default the largest power of
  // two that leaves at least two coil groups per coil of a row (each block's
  // transform groups split as rows x coil groups), times the tuner's multiple
  static int rows_per_block(const Shape &d) {
    int rpw = 1;
    while (rpw * 2 * d.cmin <= Gm::G) rpw *= 2;
    for (int m = d.rpw_mult; m > 1 && rpw < Gm::G; m /= 2) rpw *= 2;
    return rpw;
  }

  static void row_inv(const Shape &d, const float2 *t, const float2 *sens, float2 *y, const float2 *w,
                      float alpha, float beta, hipStream_t st) {
    const int rpw = rows_per_block(d);
    const int rows = d.slices * N;
    const int grid = (rows + rpw - 1) / rpw;
    if (d.cb) pf::k_row_inv<N, V, true><<<grid, Gm::THREADS, 0, st>>>(t, sens, y, w, alpha, beta, d.coils, rows, rpw, d.cb);
    else pf::k_row_inv<N, V, false><<<grid, Gm::THREADS, 0, st>>>(t, sens, y, w, alpha, beta, d.coils, rows, rpw, nullptr);
  }

  static void row_inv_fwd(const Shape &d, float2 *t, const float2 *sens, float2 *y, const float2 *w,
                          float alpha, float beta, hipStream_t st) {
    const int rpw = rows_per_block(d);
    const int rows = d.slices * N;
    const int grid = (rows + rpw - 1) / rpw;
    if (d.cb) pf::k_row_inv_fwd<N, V, true><<<grid, Gm::THREADS, 0, st>>>(t, sens, y, w, alpha, beta, d.coils, rows, rpw, d.cb);
    else pf::k_row_inv_fwd<N, V, false><<<grid, Gm::THREADS, 0, st>>>(t, sens, y, w, alpha, beta, d.coils, rows, rpw, nullptr);
  }

  // A chain of m normal applies in which apply k+1's input is apply k's output:
  //   y_k = alpha_k A^H A y_{k-1} + beta_k w_k,  y_0 = x.
  // For a 2-D mask the row passes between applies are fused (2m + 1 kernels)
  // unless the shape asks for separate passes (3m kernels).
  static void chain(const Shape &d, const float2 *sens, const uint8_t *mask, const float2 *x, int m,
                    const float *alpha, const float *beta, const float2 *const *w, float2 *const *y, float2 *t,
                    hipStream_t st, int *k_inc) {
    if (d.mask_kind != PFISTA_MASK_2D || !d.fused) {
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

  static void normal(const Shape &d, const float2 *sens, const uint8_t *mask, const float2 *x, float2 *y,
                     float alpha, const float2 *w, float beta, float2 *t, hipStream_t st, int *k_inc = nullptr) {
    if constexpr (V == 0) {
      if (d.mask_kind == PFISTA_TOEPLITZ) {
        if constexpr (N <= 256)
          ToeOps<2 * N>::normal(d, sens, reinterpret_cast<const float *>(mask), x, y, alpha, w, beta, t, st, k_inc);
        return;
      }
      if (d.mask_kind == PFISTA_MASK_1D) {
        using G1 = pf::Geo1D<N>;
        const dim3 grid(N / G1::COLS, d.slices);
        if (d.packed)
          pf::k_normal_1d<N, true><<<grid, G1::THREADS, 0, st>>>(x, sens, mask, y, w, alpha / (float)N, beta, d.coils, k_inc);
        else
          pf::k_normal_1d<N, false><<<grid, G1::THREADS, 0, st>>>(x, sens, mask, y, w, alpha / (float)N, beta, d.coils, k_inc);
        return;
      }
    }
    row_fwd(d, x, sens, t, st, k_inc);
    col<pf::COL_NORMAL>(d, t, nullptr, nullptr, mask, 1.f, 0.f, nullptr, st);
    row_inv(d, t, sens, y, w, (float)((double)alpha / ((double)N * N)), beta, st);
  }

  // FP64 partial sums the residual column pass writes: N / COLS per coil image,
  // image-major
  static int resid_per_image() { return N / Gm::COLS; }
  static int resid_blocks(const Shape &d) { return resid_per_image() * d.images; }

  // kernel passes timed by pfista_profile_normal: the three passes of one apply
  // and the fused inverse+forward row pass of the Horner chain (2-D mask), or
  // the single phase-encode pass; `pass` launches pass k alone
  static int passes(const Shape &d) {
    return d.mask_kind == PFISTA_MASK_1D ? 1 : d.mask_kind == PFISTA_TOEPLITZ ? 3 : 4;
  }
  static void pass(int k, const Shape &d, const float2 *sens, const uint8_t *mask, const float2 *x, float2 *y,
                   float alpha, const float2 *w, float beta, float2 *t, hipStream_t st) {
    if (d.mask_kind == PFISTA_TOEPLITZ) {
      if constexpr (N <= 256 && V == 0)
        ToeOps<2 * N>::pass(k, d, sens, reinterpret_cast<const float *>(mask), x, y, alpha, w, beta, t, st);
    } else if (d.mask_kind == PFISTA_MASK_1D) {
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

  static void forward(const Shape &d, const float2 *sens, const uint8_t *mask, const float2 *x,
                      float2 *kout, float2 *t, hipStream_t st) {
    row_fwd(d, x, sens, t, st);
    col<pf::COL_FWD_OUT>(d, t, nullptr, kout, mask, (float)(1.0 / N), 0.f, nullptr, st);
  }

  static void adjoint(const Shape &d, const float2 *sens, const uint8_t *mask, const float2 *kin,
                      float2 *y, float alpha, float2 *t, hipStream_t st) {
    col<pf::COL_ADJ_IN>(d, t, kin, nullptr, mask, 1.f, 0.f, nullptr, st);
    row_inv(d, t, sens, y, nullptr, (float)((double)alpha / N), 0.f, st);
  }

  // partial sums of |a M F S x - b_scale b|^2, resid_blocks(d) of them
  static void resid(const Shape &d, const float2 *sens, const uint8_t *mask, const float2 *x,
                    const float2 *b, double a, double b_scale, float2 *t, double *partials, hipStream_t st) {
    row_fwd(d, x, sens, t, st);
    col<pf::COL_RESID>(d, t, b, nullptr, mask, (float)(a / N), (float)b_scale, partials, st);
  }

  // natural -> packed coil maps of a phase-encode plan
  static void pack_1d(const Shape &d, const float2 *sens, float2 *out, hipStream_t st) {
    const dim3 grid(N / pf::Geo1D<N>::COLS, d.coils, d.slices);
    pf::k_pack_1d<N><<<grid, 256, 0, st>>>(sens, out, d.coils);
  }

  // k_dev: a valid device int; use_k != 0 takes beta = k / (k + 3) from it;
  // lam_s: per-slice thresholds (device) or nullptr for `lam`
  static void step(const Shape &d, const float2 *z, const float2 *pg, const float2 *xo, float2 *xn,
                   float2 *zn, float pg_scale, float lam, float beta, const int *k_dev, int use_k,
                   double *partials, hipStream_t st, const float *lam_s = nullptr) {
    const dim3 grid(N / 16, N / 16, d.slices);
    switch (d.haar_levels) {
      case 1: pf::k_step<1><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials, lam_s); break;
      case 2: pf::k_step<2><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials, lam_s); break;
      case 3: pf::k_step<3><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials, lam_s); break;
      default: pf::k_step<4><<<grid, 64, 0, st>>>(z, pg, xo, xn, zn, pg_scale, lam, beta, k_dev, use_k, N, partials, lam_s); break;
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

// calls the statement with NN = n and VV = v (radix-schedule variant 0 or 1)
#define PF_VCASE(NV, v, ...)                 \
  case NV: {                                 \
    constexpr int NN = NV;                   \
    if (v) {                                 \
      constexpr int VV = 1;                  \
      __VA_ARGS__;                           \
    } else {                                 \
      constexpr int VV = 0;                  \
      __VA_ARGS__;                           \
    }                                        \
  } break;
#define PF_DISPATCH_V(n, v, ...)             \
  switch (n) {                               \
    PF_VCASE(64, v, __VA_ARGS__)             \
    PF_VCASE(128, v, __VA_ARGS__)            \
    PF_VCASE(160, v, __VA_ARGS__)            \
    PF_VCASE(192, v, __VA_ARGS__)            \
    PF_VCASE(256, v, __VA_ARGS__)            \
    PF_VCASE(320, v, __VA_ARGS__)            \
    PF_VCASE(384, v, __VA_ARGS__)            \
    PF_VCASE(512, v, __VA_ARGS__)            \
    default: break;                          \
  }

const float2 *F2(const pfista_c32 *p) { return reinterpret_cast<const float2 *>(p); }
float2 *F2(pfista_c32 *p) { return reinterpret_cast<float2 *>(p); }

// y = alpha N x + beta w with the transform buffer t ([S][C][n][n], twice that
// for a Toeplitz plan)
// packed != 0: `sens` holds the packed coil maps of a phase-encode plan
void normal_op_t(const pfista_desc &d, const pfista_c32 *sens, const uint8_t *mask, const float2 *x, float2 *y,
                 float alpha, const float2 *w, float beta, float2 *t, hipStream_t st, int *k_inc = nullptr,
                 int packed = 0) {
  Shape sh = shape_of(d);
  sh.packed = packed;
  PF_DISPATCH(d.n, Ops<NN>::normal(sh, F2(sens), mask, x, y, alpha, w, beta, t, st, k_inc));
}

void normal_op(const pfista_desc &d, const pfista_c32 *sens, const uint8_t *mask, const float2 *x, float2 *y,
               float alpha, const float2 *w, float beta, void *ws, hipStream_t st, int *k_inc = nullptr) {
  normal_op_t(d, sens, mask, x, y, alpha, w, beta, at<float2>(ws, layout(d).t), st, k_inc);
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
// The applies of one gradient + polynomial chain: with `pre_x`, first the
// gradient g = inv_l A^H A pre_x - pre_w, then the Horner recursion of the
// nested form c0 I + N'(c1 I + N'(... c_d I)): h = c_d g; h = c_i g + N' h for
// i = d-1 .. 0 (the first apply folds c_d into its alpha), output in `out`.
struct Chain {
  int m = 0;
  float alpha[kMaxDegree + 1], beta[kMaxDegree + 1];
  const float2 *w[kMaxDegree + 1];
  float2 *y[kMaxDegree + 1];
  const float2 *x0 = nullptr;
};

Chain make_chain(double inv_l, const std::vector<double> &c, const float2 *pre_x, const float2 *pre_w, float2 *g,
                 float2 *out) {
  Chain ch;
  const int deg = (int)c.size() - 1;
  if (pre_x) {
    ch.alpha[ch.m] = (float)inv_l; ch.beta[ch.m] = -1.f; ch.w[ch.m] = pre_w; ch.y[ch.m] = g; ++ch.m;
  }
  for (int i = 1; i <= deg; ++i) {
    ch.alpha[ch.m] = (float)(i == 1 ? c[deg] * inv_l : inv_l);
    ch.beta[ch.m] = (float)c[deg - i];
    ch.w[ch.m] = g;
    ch.y[ch.m] = out;
    ++ch.m;
  }
  ch.x0 = pre_x ? pre_x : g;
  return ch;
}

// launch-shape candidate `cand` (see PFISTA_TUNE_CANDIDATES): radix schedule
// cand % 2, separate Horner row passes if (cand / 2) % 2, rows per coil-combine
// block times 2^(cand / 4); only 2-D masks have alternatives
int plan_candidate_ok(const pfista_desc &d, int cand) { return d.mask_kind == PFISTA_MASK_2D ? cand : 0; }

// a plan's chain of applies in the launch shape of candidate `cand`
void chain_shaped(const pfista_desc &d, int cand, const pfista_c32 *sens, const uint8_t *mask, const float2 *x0,
                  int m, const float *alpha, const float *beta, const float2 *const *w, float2 *const *y, float2 *t,
                  hipStream_t st, int *k_inc, int packed = 0) {
  cand = plan_candidate_ok(d, cand);
  Shape sh = shape_of(d);
  sh.rpw_mult = 1 << (cand / 4);
  sh.fused = (cand / 2) % 2 ? 0 : 1;
  sh.packed = packed;
  PF_DISPATCH_V(d.n, cand % 2, Ops<NN, VV>::chain(sh, F2(sens), mask, x0, m, alpha, beta, w, y, t, st, k_inc));
}

void grad_poly_op(const pfista_desc &d, const pfista_c32 *sens, const uint8_t *mask, double inv_l,
                  const std::vector<double> &c, const float2 *pre_x, const float2 *pre_w, float2 *g,
                  float2 *out, void *ws, hipStream_t st, int *k_inc, int cand = 0, int packed = 0) {
  const int deg = (int)c.size() - 1;
  const Layout L = layout(d);
  float2 *t = at<float2>(ws, L.t);
  const Chain ch = make_chain(inv_l, c, pre_x, pre_w, g, out);
  if (ch.m > 0) chain_shaped(d, cand, sens, mask, ch.x0, ch.m, ch.alpha, ch.beta, ch.w, ch.y, t, st, k_inc, packed);
  if (deg == 0 && !pre_x) pf::k_scale<<<blocks_for(L.n_img), 256, 0, st>>>(g, out, L.n_img, (float)c[0]);
}

// the plan tuner (defined with the batch tuner further down)
int tune_plan(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const std::vector<double> &c,
              double inv_l, const float2 *x0, float2 *g, float2 *pg, void *ws, hipStream_t st, int &best,
              double &best_us);

void poly_op(const pfista_desc &d, const pfista_c32 *sens, const uint8_t *mask, double inv_l,
             const std::vector<double> &c, const float2 *g, float2 *out, void *ws, hipStream_t st, int packed = 0) {
  grad_poly_op(d, sens, mask, inv_l, c, nullptr, nullptr, const_cast<float2 *>(g), out, ws, st, nullptr, 0, packed);
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

// entry checks of the calls that take packed coil maps
int check_packed_plan(const pfista_plan *p, const pfista_c32 *packed, const uint8_t *mask, const void *ws) {
  PF_TRY(check_ops(p, packed, mask, ws));
  if (p->d.mask_kind != PFISTA_MASK_1D)
    return fail(PFISTA_UNSUPPORTED, "packed coil maps exist for phase-encode plans only");
  if (p->d.slices > 0) PF_TRY(check_ptr(packed, "packed", 16));
  return PFISTA_OK;
}

// packed != 0: `sens` holds the packed coil maps of a phase-encode plan
int power_iteration_impl(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, pfista_c32 *v,
                         int iters, double *lam_max, void *ws, hipStream_t stream, int packed) {
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
    normal_op_t(p->d, sens, mask, cur, nxt, 1.f, nullptr, 0.f, at<float2>(ws, L.t), stream, nullptr, packed);
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
  if (d->mask_kind != PFISTA_MASK_2D && d->mask_kind != PFISTA_MASK_1D && d->mask_kind != PFISTA_TOEPLITZ)
    return fail(PFISTA_EINVAL, "mask_kind %d", d->mask_kind);
  // the phase-encode kernel addresses one slice's coil maps with 32-bit byte offsets
  if (d->mask_kind == PFISTA_MASK_1D && (long long)d->coils * d->n * d->n * 8 > 2147483647ll)
    return fail(PFISTA_UNSUPPORTED, "phase-encode plans need coils * n * n * 8 < 2^31 bytes per slice (got %d coils)",
                d->coils);
  if (d->mask_kind == PFISTA_TOEPLITZ && !supported_toeplitz_n(d->n))
    return fail(PFISTA_UNSUPPORTED, "Toeplitz plans need n in {64,128,160,192,256} (got %d)", d->n);
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
  return solve_ws_bytes(p->d);
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

int pfista_normal_apply_noalloc(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                                const pfista_c32 *x, pfista_c32 *y, float alpha, const pfista_c32 *w, float beta,
                                hipStream_t stream) {
  PF_TRY(check_plan(p));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(sens, "sens"));
  PF_TRY(check_ptr(mask, "mask", 1));
  PF_TRY(check_ptr(x, "x"));
  PF_TRY(check_ptr(y, "y"));
  if (w) PF_TRY(check_ptr(w, "w"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  const size_t need = L.img[0] - L.t;   // the transform buffer's section of a workspace
  if (need > PFISTA_STATIC_SCRATCH_BYTES)
    return fail(PFISTA_EINVAL, "transform buffer of %zu bytes exceeds the static scratch of %u bytes", need,
                (unsigned)PFISTA_STATIC_SCRATCH_BYTES);
  const size_t nb = L.n_img * sizeof(float2);
  if (overlaps(x, nb, y, nb)) return fail(PFISTA_EINVAL, "y overlaps x");
  if (w && w != y && overlaps(w, nb, y, nb)) return fail(PFISTA_EINVAL, "w partially overlaps y");
  float2 *t = static_cast<float2 *>(device_scratch(p->device));
  if (!t) return fail(PFISTA_EHIP, "static scratch of device %d is not set up", p->device);
  normal_op_t(p->d, sens, mask, F2(x), F2(y), alpha, w ? F2(w) : nullptr, beta, t, stream);
  return launch_status("pfista_normal_apply_noalloc");
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

int pfista_pack_coil_maps(const pfista_plan *p, const pfista_c32 *sens, pfista_c32 *packed, hipStream_t stream) {
  PF_TRY(check_plan(p));
  if (p->d.mask_kind != PFISTA_MASK_1D)
    return fail(PFISTA_UNSUPPORTED, "packed coil maps exist for phase-encode plans only");
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(sens, "sens"));
  PF_TRY(check_ptr(packed, "packed", 16));
  const Layout L = layout(p->d);
  if (L.n_coil == 0) return PFISTA_OK;
  const size_t nb = L.n_coil * sizeof(float2);
  if (overlaps(sens, nb, packed, nb)) return fail(PFISTA_EINVAL, "packed overlaps sens");
  PF_DISPATCH(p->d.n, Ops<NN>::pack_1d(shape_of(p->d), F2(sens), F2(packed), stream));
  return launch_status("pfista_pack_coil_maps");
}

int pfista_normal_apply_packed(const pfista_plan *p, const pfista_c32 *packed, const uint8_t *mask,
                               const pfista_c32 *x, pfista_c32 *y, float alpha, const pfista_c32 *w, float beta,
                               void *ws, hipStream_t stream) {
  PF_TRY(check_packed_plan(p, packed, mask, ws));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(x, "x"));
  PF_TRY(check_ptr(y, "y"));
  if (w) PF_TRY(check_ptr(w, "w"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  const size_t nb = L.n_img * sizeof(float2);
  if (overlaps(x, nb, y, nb)) return fail(PFISTA_EINVAL, "y overlaps x");
  if (w && w != y && overlaps(w, nb, y, nb)) return fail(PFISTA_EINVAL, "w partially overlaps y");
  normal_op_t(p->d, packed, mask, F2(x), F2(y), alpha, w ? F2(w) : nullptr, beta, at<float2>(ws, L.t), stream,
              nullptr, 1);
  return launch_status("pfista_normal_apply_packed");
}

int pfista_poly_apply_packed(const pfista_plan *p, const pfista_c32 *packed, const uint8_t *mask, double inv_l,
                             const double *coef, int degree, const pfista_c32 *g, pfista_c32 *out, void *ws,
                             hipStream_t stream) {
  PF_TRY(check_packed_plan(p, packed, mask, ws));
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
  poly_op(p->d, packed, mask, inv_l, c, F2(g), F2(out), ws, stream, 1);
  return launch_status("pfista_poly_apply_packed");
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
  PF_DISPATCH(p->d.n, Ops<NN>::step(shape_of(p->d), F2(z), F2(pg), F2(x_old), F2(x_new), F2(z_new), 1.f, lambda, beta_k,
                                    &ds->k, 0, partials, stream));
  const int nblk = (p->d.n / 16) * (p->d.n / 16) * p->d.slices;
  reduce(partials, nblk, 3, red, nullptr, stream);
  return launch_status("pfista_step");
}

int pfista_forward(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *x,
                   pfista_c32 *kspace, void *ws, hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.mask_kind == PFISTA_TOEPLITZ)
    return fail(PFISTA_UNSUPPORTED, "%s: Toeplitz plans have no Cartesian k-space (use pfista_nudft_*)", "pfista_forward");
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(x, "x"));
  PF_TRY(check_ptr(kspace, "kspace"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  float2 *t = at<float2>(ws, L.t);
  PF_DISPATCH(p->d.n, Ops<NN>::forward(shape_of(p->d), F2(sens), mask, F2(x), F2(kspace), t, stream));
  return launch_status("pfista_forward");
}

int pfista_adjoint(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *kspace,
                   pfista_c32 *y, float alpha, void *ws, hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.mask_kind == PFISTA_TOEPLITZ)
    return fail(PFISTA_UNSUPPORTED, "%s: Toeplitz plans have no Cartesian k-space (use pfista_nudft_*)", "pfista_adjoint");
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(kspace, "kspace"));
  PF_TRY(check_ptr(y, "y"));
  const Layout L = layout(p->d);
  if (L.n_img == 0) return PFISTA_OK;
  float2 *t = at<float2>(ws, L.t);
  PF_DISPATCH(p->d.n, Ops<NN>::adjoint(shape_of(p->d), F2(sens), mask, F2(kspace), F2(y), alpha, t, stream));
  return launch_status("pfista_adjoint");
}

int pfista_data_term(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *b,
                     const pfista_c32 *x, double inv_l, double b_scale, double *out, void *ws,
                     hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.mask_kind == PFISTA_TOEPLITZ)
    return fail(PFISTA_UNSUPPORTED, "%s: Toeplitz plans have no Cartesian k-space (use pfista_nudft_*)", "pfista_data_term");
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
  PF_DISPATCH(p->d.n, Ops<NN>::resid(shape_of(p->d), F2(sens), mask, F2(x), F2(b), std::sqrt(inv_l), b_scale, t, partials,
                                     stream));
  int cnt = 0;
  PF_DISPATCH(p->d.n, cnt = Ops<NN>::resid_blocks(shape_of(p->d)));
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
  return power_iteration_impl(p, sens, mask, v, iters, lam_max, ws, stream, 0);
}


int pfista_profile_normal(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                          const pfista_c32 *x, pfista_c32 *y, int reps, float *pass_ms, int *npasses, void *ws,
                          hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (!pass_ms || !npasses) return fail(PFISTA_EINVAL, "pass_ms/npasses is NULL");
  if (reps < 1) return fail(PFISTA_EINVAL, "reps must be >= 1");
  const pfista_desc &d = p->d;
  int np = 0;
  PF_DISPATCH(d.n, np = Ops<NN>::passes(shape_of(d)));
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
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PFISTA_EHIP, "pfista_profile_normal: event create failed");
  }
  int rc = PFISTA_OK;
  // each pass `reps` times back to back (every pass leaves valid inputs for the
  // next: the column pass is a projection, the row passes recompute their outputs)
  for (int k = 0; k < np && rc == PFISTA_OK; ++k) {
    hipError_t he = hipEventRecord(e0, stream);
    for (int r = 0; r < reps && he == hipSuccess; ++r)
      PF_DISPATCH(d.n, Ops<NN>::pass(k, shape_of(d), F2(sens), mask, F2(x), F2(y), 1.f, nullptr, 0.f, t, stream));
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
  if (prm->tune < -1 || prm->tune > PFISTA_TUNE_CANDIDATES)
    return fail(PFISTA_EINVAL, "tune outside -1..%d", PFISTA_TUNE_CANDIDATES);
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

  // ---- setup: ||b||, L, A'^H b'.  A Toeplitz plan's b is the image A^H b and
  // its ||b|| comes in the params.
  const bool toe = d.mask_kind == PFISTA_TOEPLITZ;
  double h[4] = {0, 0, 0, 0};
  double bnorm = 0.0;
  if (toe) {
    if (!(prm->bnorm > 0.0) || !std::isfinite(prm->bnorm))
      return fail(PFISTA_EINVAL, "Toeplitz plans need params.bnorm = ||b|| > 0");
    bnorm = prm->bnorm;
  } else {
    norm2_dev(F2(b), L.n_coil, partials, ds->misc, stream);
    PF_TRY(launch_status("pfista_solve(norm)"));
    PF_HIP(hipMemcpyAsync(h, ds->misc, sizeof(double), hipMemcpyDeviceToHost, stream));
    PF_HIP(hipStreamSynchronize(stream));
    bnorm = std::sqrt(h[0]);
  }
  r.bnorm = bnorm;
  // phase-encode plans: the loop (and the power iteration) read the coil maps in
  // the packed layout when the solve runs enough applies to repay the packing
  // (one read and one write of the maps, about what 11 applies save); the
  // results are the same bit for bit
  const long long solve_applies =
      (long long)prm->max_iter * (long long)c.size() + (prm->inv_l == 0.0 ? prm->power_iters : 0);
  const int packed = d.mask_kind == PFISTA_MASK_1D && solve_applies >= kPackMinApplies ? 1 : 0;
  const pfista_c32 *loop_sens = sens;
  if (packed) {
    pfista_c32 *spk = at<pfista_c32>(ws, solve_packed_off(d));
    PF_DISPATCH(d.n, Ops<NN>::pack_1d(shape_of(d), F2(sens), F2(spk), stream));
    PF_TRY(launch_status("pfista_solve(pack)"));
    loop_sens = spk;
  }
  double inv_l = prm->inv_l;
  if (inv_l == 0.0) {
    double lam = 0.0;
    PF_TRY(power_iteration_impl(p, loop_sens, mask, nullptr, prm->power_iters, &lam, ws, stream, packed));
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
  if (toe)
    pf::k_scale<<<blocks_for(L.n_img), 256, 0, stream>>>(F2(b), ahb, L.n_img, (float)(std::sqrt(inv_l) / bnorm));
  else
    PF_DISPATCH(d.n, Ops<NN>::adjoint(shape_of(d), F2(sens), mask, F2(b), ahb, (float)(std::sqrt(inv_l) / bnorm),
                                      at<float2>(ws, L.t), stream));
  if (prm->k0 == 0) {
    pf::k_fill<<<blocks_for(L.n_img), 256, 0, stream>>>(x, L.n_img, make_float2(0.f, 0.f));
    pf::k_fill<<<blocks_for(L.n_img), 256, 0, stream>>>(zb, L.n_img, make_float2(0.f, 0.f));
  }
  const int k0 = prm->k0;
  set_counter(ds, k0 - 1, stream);   // the first gradient apply advances it to k0
  PF_TRY(launch_status("pfista_solve(setup)"));

  const int deg = (int)c.size() - 1;
  const float lam = (float)prm->lambda;
  const int nstep = (d.n / 16) * (d.n / 16) * d.slices;
  // launch shape: forced, default, or tuned (cached) on the chain of this solve
  int cand = 0;
  double cand_us = 0.0;
  if (prm->tune >= 1) {
    cand = plan_candidate_ok(d, prm->tune - 1);
  } else if (prm->tune == -1 && d.mask_kind == PFISTA_MASK_2D) {
    PF_TRY(tune_plan(p, sens, mask, c, inv_l, ahb, g, pgb, ws, stream, cand, cand_us));
  }
  r.candidate = cand;
  r.tune_us = cand_us;
  auto body = [&]() {
    // g = N' z - A'^H b' then pg = p(N') g as one chain of d + 1 applies (its
    // first kernel advances the iteration counter k); then the fused step
    grad_poly_op(d, loop_sens, mask, inv_l, c, zb, ahb, g, pgb, ws, stream, &ds->k, cand, packed);
    const float2 *pg = deg == 0 ? g : pgb;
    const float pg_scale = deg == 0 ? (float)c[0] : 1.f;
    // momentum off (Algorithms 1 and 3): beta = 0, so z_(k+1) = x_(k+1)
    const int use_k = prm->momentum ? 1 : 0;
    PF_DISPATCH(d.n, Ops<NN>::step(shape_of(d), zb, pg, x, x, zb, pg_scale, lam, 0.f, &ds->k, use_k, partials, stream));
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

  // device time of the loop (set-up excluded), on the solver's stream
  struct LoopEvents {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~LoopEvents() {
      for (hipEvent_t v : e)
        if (v) (void)hipEventDestroy(v);
    }
  } lev;
  if (hipEventCreate(&lev.e[0]) != hipSuccess || hipEventCreate(&lev.e[1]) != hipSuccess) {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    return fail(PFISTA_EHIP, "pfista_solve: event create failed");
  }
  if (hipEventRecord(lev.e[0], stream) != hipSuccess) {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    return fail(PFISTA_EHIP, "pfista_solve: event record failed");
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
    if (prm->eval_objective && toe) {
      // ||A'x - b'||^2 = <x, N'x> - 2 Re <x, A'^H b'> + 1 (||b'|| = 1)
      normal_op(d, sens, mask, x, g, (float)inv_l, nullptr, 0.f, ws, stream);
      const unsigned nb = (unsigned)std::min<size_t>(kNormBlocks, (L.n_img + 255) / 256);
      pf::k_dot2<<<nb, 256, 0, stream>>>(x, g, ahb, L.n_img, partials);
      reduce(partials, (int)nb, 2, ds->misc, nullptr, stream);
      pf::k_normal_eq_data<<<1, 64, 0, stream>>>(ds->misc, ds->data);
    } else if (prm->eval_objective) {
      PF_DISPATCH(d.n, Ops<NN>::resid(shape_of(d), F2(sens), mask, x, F2(b), std::sqrt(inv_l), 1.0 / bnorm,
                                      at<float2>(ws, L.t), partials, stream));
      int cnt = 0;
      PF_DISPATCH(d.n, cnt = Ops<NN>::resid_blocks(shape_of(d)));
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
  if (done > 0) {
    float lms = 0.f;
    hipError_t te = hipEventRecord(lev.e[1], stream);
    if (te == hipSuccess) te = hipEventSynchronize(lev.e[1]);
    if (te == hipSuccess) te = hipEventElapsedTime(&lms, lev.e[0], lev.e[1]);
    if (te != hipSuccess) return fail(PFISTA_EHIP, "pfista_solve(loop timing): %s", hipGetErrorString(te));
    r.loop_ms = lms;
  }
  r.iters = done;
  r.status = status;
  r.normal_applies = (long long)done * (deg + 1);
  if (rep) *rep = r;
  return status;
}

}  // extern "C"

// ============================================================================ batches
// Slices of uneven shape, grouped by (image side, Haar levels).  A group's
// buffers are coil-image-major like a plan's, with per-slice coil counts
// described by the cb / cs tables of Shape.
struct BGroup {
  int n = 0, levels = 0;
  std::vector<int> idx;  // caller's slice indices, in group order
  std::vector<int> cb;   // first coil image of every slice, then the total
  std::vector<int> cs;   // slice (in group order) of every coil image
  int images = 0, cmin = 0, cmax = 0;
  int seg0 = 0;          // the group's first entry in the batch's per-slice sums
  size_t o_sens = 0, o_b = 0, o_t = 0, o_mask = 0, o_img[5] = {0, 0, 0, 0, 0}, o_part = 0, o_state = 0;
  size_t o_cb = 0, o_cs = 0, o_lam = 0;
  int slices() const { return (int)idx.size(); }
  size_t n_img() const { return idx.size() * (size_t)n * n; }
  size_t n_coil() const { return (size_t)images * n * n; }
};

struct pfista_batch {
  std::vector<pfista_slice_desc> sl;
  std::vector<BGroup> g;
  size_t o_norm = 0, o_npart = 0, o_seg_step = 0, o_seg_data = 0, o_scratch = 0, total = 0;
  int device = 0;
  std::string arch;
};

namespace {

// the launch shape of tuning candidate `cand` for a group; a group whose slices
// share one coil count is laid out like a plan's slices and launches without
// the coil tables (the kernels built for that case carry no table code)
Shape group_shape(const BGroup &G, void *ws, int cand) {
  const bool uniform = G.cmin == G.cmax;
  return Shape{G.slices(), G.cmax, G.images, G.levels, PFISTA_MASK_2D,
               uniform ? nullptr : at<int>(ws, G.o_cb), uniform ? nullptr : at<int>(ws, G.o_cs),
               G.cmin, 1 << (cand / 4), (cand / 2) % 2 ? 0 : 1};
}

void group_chain(const BGroup &G, const Shape &sh, int V, void *ws, const Chain &ch, hipStream_t st, int *k_inc) {
  const float2 *sens = at<float2>(ws, G.o_sens);
  const uint8_t *mask = at<uint8_t>(ws, G.o_mask);
  float2 *t = at<float2>(ws, G.o_t);
  PF_DISPATCH_V(G.n, V, Ops<NN, VV>::chain(sh, sens, mask, ch.x0, ch.m, ch.alpha, ch.beta, ch.w, ch.y, t, st, k_inc));
}

// architecture name of a device without its feature suffix ("gfx950")
std::mutex g_arch_mu;
std::vector<std::string> g_arch;

std::string device_arch(int dev) {
  std::lock_guard<std::mutex> lk(g_arch_mu);
  if ((int)g_arch.size() <= dev) g_arch.resize(dev + 1);
  if (g_arch[dev].empty()) {
    hipDeviceProp_t prop;
    std::string a = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      a = prop.gcnArchName;
      const size_t colon = a.find(':');
      if (colon != std::string::npos) a.resize(colon);
    }
    g_arch[dev] = a;
  }
  return g_arch[dev];
}

// ---- tuner cache: per device architecture and plan or group signature;
// optionally persisted as "key candidate microseconds" lines in $PFISTA_TUNE_CACHE
std::mutex g_tune_mu;
std::vector<std::pair<std::string, std::pair<int, double>>> g_tune;
bool g_tune_read = false;

std::string tune_key(const std::string &arch, const BGroup &G, int deg) {
  char buf[320];
  snprintf(buf, sizeof buf, "%s|n%d|L%d|s%d|ci%d|c%d-%d|d%d", arch.c_str(), G.n, G.levels, G.slices(), G.images,
           G.cmin, G.cmax, deg);
  return buf;
}

void tune_read_file() {
  g_tune_read = true;
  const char *path = getenv("PFISTA_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char key[320];
  int cand = 0;
  double us = 0.0;
  while (fscanf(f, "%319s %d %lf", key, &cand, &us) == 3)
    if (cand >= 0 && cand < PFISTA_TUNE_CANDIDATES) g_tune.push_back({key, {cand, us}});
  fclose(f);
}

bool tune_lookup(const std::string &key, int &cand, double &us) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_read) tune_read_file();
  for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
    if (it->first == key) {
      cand = it->second.first;
      us = it->second.second;
      return true;
    }
  return false;
}

void tune_store(const std::string &key, int cand, double us) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.push_back({key, {cand, us}});
  const char *path = getenv("PFISTA_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE *f = fopen(path, "a")) {
    fprintf(f, "%s %d %.3f\n", key.c_str(), cand, us);
    fclose(f);
  }
}

// Time one gradient + polynomial chain of the group for every distinct
// candidate shape (one warm-up, then three timed chains) and return the fastest.
int tune_group(const BGroup &G, void *ws, const std::vector<double> &c, hipStream_t st, int &best, double &best_us) {
  float2 *ahb = at<float2>(ws, G.o_img[0]), *g = at<float2>(ws, G.o_img[1]), *pg = at<float2>(ws, G.o_img[2]);
  const Chain ch = make_chain(1.0, c, ahb, ahb, g, pg);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PF_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PFISTA_EHIP, "tuner: event create failed");
  }
  best = 0;
  best_us = 0.0;
  int rc = PFISTA_OK;
  std::vector<int> seen;
  for (int k = 0; k < PFISTA_TUNE_CANDIDATES && rc == PFISTA_OK; ++k) {
    const Shape sh = group_shape(G, ws, k);
    const int V = k % 2;
    int rpw = 0;
    PF_DISPATCH_V(G.n, V, rpw = Ops<NN, VV>::rows_per_block(sh));
    const int sig = (V * 2 + sh.fused) * 1024 + rpw;
    if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
    seen.push_back(sig);
    group_chain(G, sh, V, ws, ch, st, nullptr);
    hipError_t he = hipEventRecord(e0, st);
    for (int r = 0; r < 3 && he == hipSuccess; ++r) group_chain(G, sh, V, ws, ch, st, nullptr);
    if (he == hipSuccess) he = hipEventRecord(e1, st);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) {
      rc = fail(PFISTA_EHIP, "tuner: %s", hipGetErrorString(he));
      break;
    }
    rc = launch_status("tuner");
    const double us = 1e3 * ms / 3.0;
    if (seen.size() == 1 || us < best_us) {
      best = k;
      best_us = us;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// Plan solves: time one gradient + polynomial chain from x0 for every distinct
// candidate (one warm-up, three timed), cached per architecture and plan shape.
int tune_plan(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const std::vector<double> &c,
              double inv_l, const float2 *x0, float2 *g, float2 *pg, void *ws, hipStream_t st, int &best,
              double &best_us) {
  const pfista_desc &d = p->d;
  const int deg = (int)c.size() - 1;
  char key[320];
  snprintf(key, sizeof key, "%s|plan|n%d|s%d|c%d|L%d|d%d", device_arch(p->device).c_str(), d.n, d.slices, d.coils,
           d.haar_levels, deg);
  if (tune_lookup(key, best, best_us)) return PFISTA_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PF_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PFISTA_EHIP, "tuner: event create failed");
  }
  best = 0;
  best_us = 0.0;
  int rc = PFISTA_OK;
  std::vector<int> seen;
  for (int k = 0; k < PFISTA_TUNE_CANDIDATES && rc == PFISTA_OK; ++k) {
    Shape sh = shape_of(d);
    sh.rpw_mult = 1 << (k / 4);
    sh.fused = (k / 2) % 2 ? 0 : 1;
    int rpw = 0;
    PF_DISPATCH_V(d.n, k % 2, rpw = Ops<NN, VV>::rows_per_block(sh));
    const int sig = ((k % 2) * 2 + sh.fused) * 1024 + rpw;
    if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
    seen.push_back(sig);
    grad_poly_op(d, sens, mask, inv_l, c, x0, x0, g, pg, ws, st, nullptr, k);
    hipError_t he = hipEventRecord(e0, st);
    for (int r = 0; r < 3 && he == hipSuccess; ++r) grad_poly_op(d, sens, mask, inv_l, c, x0, x0, g, pg, ws, st, nullptr, k);
    if (he == hipSuccess) he = hipEventRecord(e1, st);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) {
      rc = fail(PFISTA_EHIP, "tuner: %s", hipGetErrorString(he));
      break;
    }
    rc = launch_status("tuner");
    const double us = 1e3 * ms / 3.0;
    if (seen.size() == 1 || us < best_us) {
      best = k;
      best_us = us;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == PFISTA_OK) tune_store(key, best, best_us);
  return rc;
}

int check_batch_params(const pfista_batch_params *prm, std::vector<double> &c) {
  if (!prm) return fail(PFISTA_EINVAL, "params is NULL");
  if (prm->max_iter < 0) return fail(PFISTA_EINVAL, "max_iter < 0");
  if (prm->check_every < 1 || prm->check_every > 4096) return fail(PFISTA_EINVAL, "check_every outside 1..4096");
  if (prm->tune < -1 || prm->tune > PFISTA_TUNE_CANDIDATES)
    return fail(PFISTA_EINVAL, "tune outside -1..%d", PFISTA_TUNE_CANDIDATES);
  if (prm->streams < 1 || prm->streams > 64) return fail(PFISTA_EINVAL, "streams outside 1..64");
  if (prm->graph_iters < 0) return fail(PFISTA_EINVAL, "graph_iters < 0");
  if (prm->coef) {
    if (prm->degree < 0 || prm->degree > kMaxDegree) return fail(PFISTA_UNSUPPORTED, "degree %d", prm->degree);
    c.assign(prm->coef, prm->coef + prm->degree + 1);
    return PFISTA_OK;
  }
  return l2_coefficients(prm->degree, c);
}

// Streams, events and graph of one batch solve, released on every exit path.
struct BatchRun {
  std::vector<hipStream_t> br;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipGraphExec_t gexec = nullptr;
  ~BatchRun() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (size_t i = 1; i < br.size(); ++i)
      if (br[i] && br[i] != br[0]) (void)hipStreamDestroy(br[i]);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
};

}  // namespace

extern "C" {

int pfista_batch_create(pfista_batch **out, const pfista_slice_desc *slices, int count, size_t chunk_bytes) {
  if (!out) return fail(PFISTA_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 0) return fail(PFISTA_EINVAL, "count < 0");
  if (count > 0 && !slices) return fail(PFISTA_EINVAL, "slices is NULL");
  for (int s = 0; s < count; ++s) {
    const pfista_slice_desc &d = slices[s];
    if (!supported_n(d.n)) return fail(PFISTA_UNSUPPORTED, "slice %d: image side %d not supported", s, d.n);
    if (d.coils < 1) return fail(PFISTA_EINVAL, "slice %d: coils must be >= 1", s);
    if (d.haar_levels < 1 || d.haar_levels > 4)
      return fail(PFISTA_UNSUPPORTED, "slice %d: haar_levels %d outside 1..4", s, d.haar_levels);
  }
  PF_TRY(ensure_twiddles());
  pfista_batch *b = new (std::nothrow) pfista_batch;
  if (!b) return fail(PFISTA_EINVAL, "out of host memory");
  b->sl.assign(slices, slices + count);
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return fail(PFISTA_EHIP, "hipGetDevice failed");
  }
  b->arch = device_arch(b->device);
  // groups in ascending (n, levels), slices in caller order inside a group
  std::vector<int> order(count);
  for (int s = 0; s < count; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return slices[a].n != slices[c].n ? slices[a].n < slices[c].n : slices[a].haar_levels < slices[c].haar_levels;
  });
  for (int s : order) {
    const pfista_slice_desc &d = slices[s];
    const size_t bytes = (size_t)d.coils * d.n * d.n * sizeof(float2);
    if (b->g.empty() || b->g.back().n != d.n || b->g.back().levels != d.haar_levels ||
        (chunk_bytes > 0 && b->g.back().n_coil() * sizeof(float2) + bytes > chunk_bytes)) {
      BGroup G;
      G.n = d.n;
      G.levels = d.haar_levels;
      G.cb.push_back(0);
      G.cmin = d.coils;
      G.cmax = d.coils;
      b->g.push_back(G);
    }
    BGroup &G = b->g.back();
    for (int c = 0; c < d.coils; ++c) G.cs.push_back(G.slices());
    G.idx.push_back(s);
    G.images += d.coils;
    G.cb.push_back(G.images);
    G.cmin = std::min(G.cmin, d.coils);
    G.cmax = std::max(G.cmax, d.coils);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  int seg = 0;
  size_t scratch = 16;
  for (BGroup &G : b->g) {
    if (G.images > 65535) {
      delete b;
      return fail(PFISTA_UNSUPPORTED, "group of side %d holds %d coil images (> 65535)", G.n, G.images);
    }
    G.seg0 = seg;
    seg += G.slices();
    G.o_sens = take(G.n_coil() * sizeof(float2));
    G.o_b = take(G.n_coil() * sizeof(float2));
    G.o_t = take(G.n_coil() * sizeof(float2));
    G.o_mask = take(G.n_img());
    for (int i = 0; i < 5; ++i) G.o_img[i] = take(G.n_img() * sizeof(float2));
    int rpi = 0;
    for (int v = 0; v < pf::kVariants; ++v) {
      int r = 0;
      PF_DISPATCH_V(G.n, v, r = Ops<NN, VV>::resid_per_image());
      rpi = std::max(rpi, r);
    }
    const size_t n_part = std::max<size_t>({(size_t)3 * G.slices() * (G.n / 16) * (G.n / 16),
                                            (size_t)rpi * G.images, (size_t)16});
    G.o_part = take(n_part * sizeof(double));
    G.o_state = take(sizeof(DevState));
    G.o_cb = take(G.cb.size() * sizeof(int));
    G.o_cs = take(G.cs.size() * sizeof(int));
    G.o_lam = take(G.idx.size() * sizeof(float));
    for (int s : G.idx) {
      const pfista_desc d1{G.n, slices[s].coils, 1, G.levels, PFISTA_MASK_2D};
      scratch = std::max(scratch, layout(d1).total);
    }
  }
  b->o_norm = take((size_t)count * sizeof(double));
  b->o_npart = take((size_t)kNormBlocks * sizeof(double));
  b->o_seg_step = take((size_t)count * 3 * sizeof(double));
  b->o_seg_data = take((size_t)count * sizeof(double));
  b->o_scratch = take(scratch);
  b->total = off;
  *out = b;
  return PFISTA_OK;
}

void pfista_batch_destroy(pfista_batch *b) { delete b; }

size_t pfista_batch_workspace_bytes(const pfista_batch *b) { return b ? b->total : 0; }

int pfista_batch_groups(const pfista_batch *b) { return b ? (int)b->g.size() : 0; }

int pfista_batch_solve(const pfista_batch *b, const pfista_c32 *const *sens, const uint8_t *const *mask,
                       const pfista_c32 *const *kspace, const double *lambda, const double *inv_l,
                       const pfista_batch_params *prm, pfista_c32 *const *x_out, pfista_slice_report *slice_rep,
                       pfista_group_report *group_rep, pfista_batch_report *rep, void *ws, hipStream_t stream) {
  if (!b) return fail(PFISTA_EINVAL, "batch is NULL");
  PF_TRY(check_device(b->device));
  std::vector<double> c;
  PF_TRY(check_batch_params(prm, c));
  const int count = (int)b->sl.size();
  pfista_batch_report r{};
  r.status = PFISTA_OK;
  if (count == 0) {
    if (rep) *rep = r;
    return PFISTA_OK;
  }
  if (!sens || !mask || !kspace || !lambda || !x_out) return fail(PFISTA_EINVAL, "a per-slice pointer array is NULL");
  PF_TRY(check_ptr(ws, "ws", 16));
  bool need_power = false;
  for (int s = 0; s < count; ++s) {
    char nm[64];
    snprintf(nm, sizeof nm, "sens[%d]", s);
    PF_TRY(check_ptr(sens[s], nm));
    snprintf(nm, sizeof nm, "mask[%d]", s);
    PF_TRY(check_ptr(mask[s], nm, 1));
    snprintf(nm, sizeof nm, "kspace[%d]", s);
    PF_TRY(check_ptr(kspace[s], nm));
    snprintf(nm, sizeof nm, "x_out[%d]", s);
    PF_TRY(check_ptr(x_out[s], nm));
    if (!(lambda[s] >= 0.0) || !std::isfinite(lambda[s])) return fail(PFISTA_EINVAL, "lambda[%d] must be finite and >= 0", s);
    const double il = inv_l ? inv_l[s] : 0.0;
    if (!(il >= 0.0) || !std::isfinite(il)) return fail(PFISTA_EINVAL, "inv_l[%d] must be finite and >= 0", s);
    need_power = need_power || il == 0.0;
  }
  if (need_power && prm->power_iters < 1) return fail(PFISTA_EINVAL, "estimating inv_l needs power_iters >= 1");
  const int dev = b->device;   // current (checked above)
  const int deg = (int)c.size() - 1;
  const int ng = (int)b->g.size();

  // ---- setup: ||b_s||, L_s, normalised copies, A'^H b'
  double *norm = at<double>(ws, b->o_norm);
  double *npart = at<double>(ws, b->o_npart);
  for (int s = 0; s < count; ++s)
    norm2_dev(F2(kspace[s]), (size_t)b->sl[s].coils * b->sl[s].n * b->sl[s].n, npart, norm + s, stream);
  PF_TRY(launch_status("pfista_batch_solve(norm)"));
  std::vector<double> il(count), bn(count);
  for (int s = 0; s < count; ++s) {
    il[s] = inv_l ? inv_l[s] : 0.0;
    if (il[s] == 0.0) {
      const pfista_slice_desc &d = b->sl[s];
      pfista_plan tmp;
      tmp.d = pfista_desc{d.n, d.coils, 1, d.haar_levels, PFISTA_MASK_2D};
      tmp.device = dev;
      double lam = 0.0;
      PF_TRY(pfista_power_iteration(&tmp, sens[s], mask[s], nullptr, prm->power_iters, &lam,
                                    at<void>(ws, b->o_scratch), stream));
      if (!(lam > 0.0)) return fail(PFISTA_EINVAL, "slice %d: power iteration gave %g", s, lam);
      il[s] = 1.0 / (1.01 * lam);
    }
  }
  PF_HIP(hipMemcpyAsync(bn.data(), norm, count * sizeof(double), hipMemcpyDeviceToHost, stream));
  PF_HIP(hipStreamSynchronize(stream));
  for (int s = 0; s < count; ++s) bn[s] = std::sqrt(bn[s]);

  std::vector<std::vector<float>> lam_h(ng);
  for (int gi = 0; gi < ng; ++gi) {
    const BGroup &G = b->g[gi];
    const size_t nn = (size_t)G.n * G.n;
    for (int s : G.idx) lam_h[gi].push_back((float)lambda[s]);
    PF_HIP(hipMemcpyAsync(at<int>(ws, G.o_cb), G.cb.data(), G.cb.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    PF_HIP(hipMemcpyAsync(at<int>(ws, G.o_cs), G.cs.data(), G.cs.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    PF_HIP(hipMemcpyAsync(at<float>(ws, G.o_lam), lam_h[gi].data(), lam_h[gi].size() * sizeof(float),
                          hipMemcpyHostToDevice, stream));
    float2 *sg = at<float2>(ws, G.o_sens), *bg = at<float2>(ws, G.o_b);
    uint8_t *mg = at<uint8_t>(ws, G.o_mask);
    for (int j = 0; j < G.slices(); ++j) {
      const int s = G.idx[j];
      const size_t nc = (size_t)b->sl[s].coils * nn;
      pf::k_scale<<<blocks_for(nc), 256, 0, stream>>>(F2(sens[s]), sg + (size_t)G.cb[j] * nn, nc,
                                                      (float)std::sqrt(il[s]));
      pf::k_scale<<<blocks_for(nc), 256, 0, stream>>>(F2(kspace[s]), bg + (size_t)G.cb[j] * nn, nc,
                                                      bn[s] > 0.0 ? (float)(1.0 / bn[s]) : 0.f);
      PF_HIP(hipMemcpyAsync(mg + (size_t)j * nn, mask[s], nn, hipMemcpyDeviceToDevice, stream));
    }
    const Shape sh0 = group_shape(G, ws, 0);
    PF_DISPATCH_V(G.n, 0, Ops<NN, VV>::adjoint(sh0, sg, mg, bg, at<float2>(ws, G.o_img[0]), 1.f,
                                               at<float2>(ws, G.o_t), stream));
    pf::k_fill<<<blocks_for(G.n_img()), 256, 0, stream>>>(at<float2>(ws, G.o_img[3]), G.n_img(), make_float2(0.f, 0.f));
    pf::k_fill<<<blocks_for(G.n_img()), 256, 0, stream>>>(at<float2>(ws, G.o_img[4]), G.n_img(), make_float2(0.f, 0.f));
    set_counter(at<DevState>(ws, G.o_state), -1, stream);   // the first gradient apply advances it to 0
  }
  PF_TRY(launch_status("pfista_batch_solve(setup)"));
  // the per-group tables were copied from host vectors: let the copies land
  PF_HIP(hipStreamSynchronize(stream));

  // ---- launch shape per group
  std::vector<int> cand(ng, 0);
  std::vector<double> cand_us(ng, 0.0);
  for (int gi = 0; gi < ng; ++gi) {
    if (prm->tune >= 1) {
      cand[gi] = prm->tune - 1;
    } else if (prm->tune == -1) {
      const std::string key = tune_key(b->arch, b->g[gi], deg);
      if (!tune_lookup(key, cand[gi], cand_us[gi])) {
        PF_TRY(tune_group(b->g[gi], ws, c, stream, cand[gi], cand_us[gi]));
        tune_store(key, cand[gi], cand_us[gi]);
      }
    }
  }
  std::vector<Shape> shp(ng);
  for (int gi = 0; gi < ng; ++gi) shp[gi] = group_shape(b->g[gi], ws, cand[gi]);

  // ---- branches: groups spread by longest-processing-time on coil-image pixels
  BatchRun run;
  const int nb = std::min(prm->streams, ng);
  run.br.assign(nb, nullptr);   // slots 1.. are owned and destroyed by BatchRun
  run.br[0] = stream;
  std::vector<int> branch(ng, 0);
  if (nb > 1) {
    for (int i = 1; i < nb; ++i) PF_HIP(hipStreamCreateWithFlags(&run.br[i], hipStreamNonBlocking));
    PF_HIP(hipEventCreateWithFlags(&run.fork, hipEventDisableTiming));
    run.join.assign(nb, nullptr);
    for (int i = 1; i < nb; ++i) PF_HIP(hipEventCreateWithFlags(&run.join[i], hipEventDisableTiming));
    std::vector<int> ord(ng);
    for (int gi = 0; gi < ng; ++gi) ord[gi] = gi;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int q) { return b->g[a].n_coil() > b->g[q].n_coil(); });
    std::vector<double> load(nb, 0.0);
    for (int gi : ord) {
      const int tgt = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      branch[gi] = tgt;
      load[tgt] += (double)b->g[gi].n_coil();
    }
  }

  const int use_k = prm->momentum ? 1 : 0;
  auto body = [&]() -> hipError_t {
    hipError_t he = hipSuccess;
    if (nb > 1) {
      he = hipEventRecord(run.fork, stream);
      for (int i = 1; i < nb && he == hipSuccess; ++i) he = hipStreamWaitEvent(run.br[i], run.fork, 0);
      if (he != hipSuccess) return he;
    }
    for (int gi = 0; gi < ng; ++gi) {
      const BGroup &G = b->g[gi];
      hipStream_t st = run.br[branch[gi]];
      float2 *ahb = at<float2>(ws, G.o_img[0]), *g = at<float2>(ws, G.o_img[1]), *pg = at<float2>(ws, G.o_img[2]);
      float2 *x = at<float2>(ws, G.o_img[3]), *z = at<float2>(ws, G.o_img[4]);
      DevState *ds = at<DevState>(ws, G.o_state);
      const Chain ch = make_chain(1.0, c, z, ahb, g, pg);
      const int V = cand[gi] % 2;
      group_chain(G, shp[gi], V, ws, ch, st, &ds->k);
      const float2 *pgp = deg == 0 ? g : pg;
      const float pg_scale = deg == 0 ? (float)c[0] : 1.f;
      PF_DISPATCH_V(G.n, V, Ops<NN, VV>::step(shp[gi], z, pgp, x, x, z, pg_scale, 0.f, 0.f, &ds->k, use_k,
                                              at<double>(ws, G.o_part), st, at<float>(ws, G.o_lam)));
    }
    if (nb > 1) {
      for (int i = 1; i < nb && he == hipSuccess; ++i) he = hipEventRecord(run.join[i], run.br[i]);
      for (int i = 1; i < nb && he == hipSuccess; ++i) he = hipStreamWaitEvent(stream, run.join[i], 0);
    }
    return he;
  };

  int gunroll = 0;
  if (prm->graph_iters > 0 && stream != nullptr && prm->max_iter > 0) {
    gunroll = std::min(prm->graph_iters, prm->check_every);
    hipGraph_t graph = nullptr;
    PF_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    hipError_t be = hipSuccess;
    for (int i = 0; i < gunroll && be == hipSuccess; ++i) be = body();
    hipError_t ce = hipStreamEndCapture(stream, &graph);
    if (be != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(PFISTA_EHIP, "graph capture: %s", hipGetErrorString(be));
    }
    if (ce != hipSuccess) return fail(PFISTA_EHIP, "graph capture: %s", hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&run.gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(PFISTA_EHIP, "graph instantiate: %s", hipGetErrorString(ie));
  }

  double *seg_step = at<double>(ws, b->o_seg_step), *seg_data = at<double>(ws, b->o_seg_data);
  std::vector<double> hs((size_t)count * 3), hd(count, 0.0);
  std::vector<pfista_slice_report> sr(count);
  for (int s = 0; s < count; ++s) {
    sr[s] = pfista_slice_report{NAN, 0.0, 0.0, il[s], bn[s]};
  }
  int done = 0, status = PFISTA_OK;
  while (done < prm->max_iter) {
    const int chunk = std::min(prm->check_every, prm->max_iter - done);
    int left = chunk;
    if (run.gexec) {
      while (left >= gunroll) {
        hipError_t le = hipGraphLaunch(run.gexec, stream);
        if (le != hipSuccess) return fail(PFISTA_EHIP, "graph launch: %s", hipGetErrorString(le));
        left -= gunroll;
      }
    }
    for (; left > 0; --left) {
      hipError_t be = body();
      if (be != hipSuccess) return fail(PFISTA_EHIP, "pfista_batch_solve(loop): %s", hipGetErrorString(be));
    }
    done += chunk;
    // per-slice FP64 sums of the chunk's last step, and optionally the data term
    for (int gi = 0; gi < ng; ++gi) {
      const BGroup &G = b->g[gi];
      double *part = at<double>(ws, G.o_part);
      pf::k_reduce_seg<<<G.slices(), 64, 0, stream>>>(part, nullptr, (G.n / 16) * (G.n / 16), 3,
                                                      seg_step + 3 * (size_t)G.seg0);
      if (prm->eval_objective) {
        const int V = cand[gi] % 2;
        int rpi = 0;
        PF_DISPATCH_V(G.n, V, rpi = Ops<NN, VV>::resid_per_image());
        PF_DISPATCH_V(G.n, V, Ops<NN, VV>::resid(shp[gi], at<float2>(ws, G.o_sens), at<uint8_t>(ws, G.o_mask),
                                                 at<float2>(ws, G.o_img[3]), at<float2>(ws, G.o_b), 1.0, 1.0,
                                                 at<float2>(ws, G.o_t), part, stream));
        pf::k_reduce_seg<<<G.slices(), 64, 0, stream>>>(part, at<int>(ws, G.o_cb), rpi, 1, seg_data + G.seg0);
      }
    }
    PF_TRY(launch_status("pfista_batch_solve(check)"));
    PF_HIP(hipMemcpyAsync(hs.data(), seg_step, hs.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    if (prm->eval_objective)
      PF_HIP(hipMemcpyAsync(hd.data(), seg_data, hd.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    PF_HIP(hipStreamSynchronize(stream));
    bool all_tol = prm->tol > 0;
    bool bad = false;
    for (const BGroup &G : b->g)
      for (int j = 0; j < G.slices(); ++j) {
        const int s = G.idx[j];
        const size_t q = (size_t)G.seg0 + j;
        const double l1 = hs[3 * q], dx2 = hs[3 * q + 1], xn2 = hs[3 * q + 2];
        sr[s].l1 = l1;
        sr[s].rel_change = xn2 > 0 ? std::sqrt(dx2 / xn2) : 0.0;
        if (prm->eval_objective) sr[s].objective = 0.5 * hd[q] + lambda[s] * l1;
        bad = bad || !std::isfinite(l1) || !std::isfinite(dx2) || !std::isfinite(xn2) ||
              (prm->eval_objective && (!std::isfinite(sr[s].objective) || sr[s].objective > 5.0));
        all_tol = all_tol && sr[s].rel_change <= prm->tol;
      }
    if (bad) {
      status = PFISTA_DIVERGED;
      fail(PFISTA_DIVERGED, "a slice diverged after %d iterations", done);
      break;
    }
    if (all_tol) break;
  }

  // ---- outputs
  for (const BGroup &G : b->g) {
    const size_t nn = (size_t)G.n * G.n;
    for (int j = 0; j < G.slices(); ++j)
      PF_HIP(hipMemcpyAsync(x_out[G.idx[j]], at<float2>(ws, G.o_img[3]) + (size_t)j * nn, nn * sizeof(float2),
                            hipMemcpyDeviceToDevice, stream));
  }
  PF_HIP(hipStreamSynchronize(stream));
  if (slice_rep)
    for (int s = 0; s < count; ++s) slice_rep[s] = sr[s];
  if (group_rep)
    for (int gi = 0; gi < ng; ++gi) {
      const BGroup &G = b->g[gi];
      group_rep[gi] = pfista_group_report{G.n, G.levels, G.slices(), G.images, cand[gi], cand_us[gi]};
    }
  r.iters = done;
  r.status = status;
  r.normal_applies = (long long)done * (deg + 1);
  if (rep) *rep = r;
  return status;
}

}  // extern "C"

// ============================================================================ unrolled iterations
namespace {

struct ULayout {
  Layout base;        // the plan's workspace (t, five images, partials, state)
  size_t seg = 0;     // segment store: z_k, g_k, pg_k for ckpt_every steps
  size_t q = 0;       // q_0 .. q_d, contiguous (stride n_img)
  size_t pv = 0, xb = 0, zb = 0, zb2 = 0, x = 0, z = 0, cpart = 0, grad = 0, total = 0;
  int ck = 1, nck = 1, ncomb = 1;
};

int check_unroll(const pfista_unroll_params *prm, std::vector<double> &c) {
  if (!prm) return fail(PFISTA_EINVAL, "params is NULL");
  if (prm->iters < 1) return fail(PFISTA_EINVAL, "iters must be >= 1");
  if (prm->ckpt_every < 1) return fail(PFISTA_EINVAL, "ckpt_every must be >= 1");
  if (!(prm->lambda >= 0.0) || !std::isfinite(prm->lambda)) return fail(PFISTA_EINVAL, "lambda must be finite and >= 0");
  if (!(prm->inv_l > 0.0) || !std::isfinite(prm->inv_l)) return fail(PFISTA_EINVAL, "inv_l must be finite and > 0");
  if (prm->tune < -1 || prm->tune > PFISTA_TUNE_CANDIDATES)
    return fail(PFISTA_EINVAL, "tune outside -1..%d", PFISTA_TUNE_CANDIDATES);
  if (prm->coef) {
    if (prm->degree < 0 || prm->degree > kMaxDegree) return fail(PFISTA_UNSUPPORTED, "degree %d", prm->degree);
    c.assign(prm->coef, prm->coef + prm->degree + 1);
    return PFISTA_OK;
  }
  return l2_coefficients(prm->degree, c);
}

ULayout ulayout(const pfista_desc &d, const pfista_unroll_params *prm) {
  ULayout U;
  U.base = layout(d);
  const int deg = prm->coef ? prm->degree : std::max(0, std::min(prm->degree, kMaxDegree));
  U.ck = std::max(1, std::min(prm->ckpt_every, prm->iters));
  U.nck = (prm->iters + U.ck - 1) / U.ck;
  const size_t img = U.base.n_img * sizeof(float2);
  size_t off = U.base.total;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  U.seg = take(3 * (size_t)U.ck * img);
  U.q = take((size_t)(deg + 1) * img);
  U.pv = take(img);
  U.xb = take(img);
  U.zb = take(img);
  U.zb2 = take(img);
  U.x = take(img);
  U.z = take(img);
  U.ncomb = (int)std::max<size_t>(1, std::min<size_t>(256, (U.base.n_img + 255) / 256));
  U.cpart = take((size_t)U.ncomb * (deg + 1) * sizeof(double));
  U.grad = take((size_t)(deg + 2) * sizeof(double));
  U.total = off;
  return U;
}

size_t ckpt_bytes(const pfista_desc &d, const ULayout &U) {
  return (size_t)(1 + 2 * U.nck) * layout(d).n_img * sizeof(float2);
}


// launch shape of the unrolled passes: params.tune as in pfista_params (the tuner
// times chains from the image `x0` into the scratch images g, pg)
int unroll_candidate(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const std::vector<double> &c,
                     double inv_l, int tune, const float2 *x0, float2 *g, float2 *pg, void *ws, hipStream_t st,
                     int &cand) {
  cand = 0;
  if (tune >= 1) {
    cand = plan_candidate_ok(p->d, tune - 1);
  } else if (tune == -1 && p->d.mask_kind == PFISTA_MASK_2D) {
    double us = 0.0;
    PF_TRY(tune_plan(p, sens, mask, c, inv_l, x0, g, pg, ws, st, cand, us));
  }
  return PFISTA_OK;
}

// One forward step of Algorithm 4 from (x, z): writes g and pg, then x, z.
void unroll_step(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const std::vector<double> &c,
                 double inv_l, float lam, int use_k, const float2 *a, float2 *x, float2 *z, float2 *g, float2 *pg,
                 void *ws, hipStream_t st, int cand) {
  const Layout L = layout(p->d);
  DevState *ds = at<DevState>(ws, L.state);
  const int deg = (int)c.size() - 1;
  grad_poly_op(p->d, sens, mask, inv_l, c, z, a, g, pg, ws, st, &ds->k, cand);
  if (deg == 0) pf::k_scale<<<blocks_for(L.n_img), 256, 0, st>>>(g, pg, L.n_img, (float)c[0]);
  PF_DISPATCH(p->d.n, Ops<NN>::step(shape_of(p->d), z, pg, x, x, z, 1.f, lam, 0.f, &ds->k, use_k,
                                    at<double>(ws, L.partials), st));
}

}  // namespace

extern "C" {

size_t pfista_unroll_ckpt_bytes(const pfista_plan *p, const pfista_unroll_params *prm) {
  std::vector<double> c;
  if (!p || check_unroll(prm, c) != PFISTA_OK) return 0;
  pfista_unroll_params q = *prm;
  q.degree = (int)c.size() - 1;
  q.coef = c.data();
  return ckpt_bytes(p->d, ulayout(p->d, &q));
}

size_t pfista_unroll_workspace_bytes(const pfista_plan *p, const pfista_unroll_params *prm) {
  std::vector<double> c;
  if (!p || check_unroll(prm, c) != PFISTA_OK) return 0;
  pfista_unroll_params q = *prm;
  q.degree = (int)c.size() - 1;
  q.coef = c.data();
  return ulayout(p->d, &q).total;
}

int pfista_unroll_forward(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask, const pfista_c32 *b,
                          const pfista_unroll_params *prm, pfista_c32 *x_out, void *ckpt, void *ws,
                          hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.mask_kind == PFISTA_TOEPLITZ) return fail(PFISTA_UNSUPPORTED, "pfista_unroll_forward: Cartesian plans only");
  std::vector<double> c;
  PF_TRY(check_unroll(prm, c));
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(b, "b"));
  PF_TRY(check_ptr(x_out, "x_out"));
  PF_TRY(check_ptr(ckpt, "ckpt", 16));
  pfista_unroll_params q = *prm;
  q.degree = (int)c.size() - 1;
  q.coef = c.data();
  const ULayout U = ulayout(p->d, &q);
  const size_t n = U.base.n_img;
  if (n == 0) return PFISTA_OK;
  DevState *ds = at<DevState>(ws, U.base.state);
  double *partials = at<double>(ws, U.base.partials);
  // ||b|| (the normalisation of Section 3), then a = A'^H b'
  norm2_dev(F2(b), U.base.n_coil, partials, ds->misc, stream);
  PF_TRY(launch_status("pfista_unroll_forward(norm)"));
  double h = 0.0;
  PF_HIP(hipMemcpyAsync(&h, ds->misc, sizeof(double), hipMemcpyDeviceToHost, stream));
  PF_HIP(hipStreamSynchronize(stream));
  const double bnorm = std::sqrt(h);
  float2 *ck = static_cast<float2 *>(ckpt);
  float2 *a = ck;
  float2 *x = at<float2>(ws, U.x), *z = at<float2>(ws, U.z);
  const double il = prm->inv_l;
  PF_DISPATCH(p->d.n, Ops<NN>::adjoint(shape_of(p->d), F2(sens), mask, F2(b), a,
                                       bnorm > 0.0 ? (float)(std::sqrt(il) / bnorm) : 0.f, at<float2>(ws, U.base.t),
                                       stream));
  int cand = 0;
  PF_TRY(unroll_candidate(p, sens, mask, c, il, prm->tune, a, at<float2>(ws, U.base.img[1]),
                          at<float2>(ws, U.base.img[2]), ws, stream, cand));
  pf::k_fill<<<blocks_for(n), 256, 0, stream>>>(x, n, make_float2(0.f, 0.f));
  pf::k_fill<<<blocks_for(n), 256, 0, stream>>>(z, n, make_float2(0.f, 0.f));
  set_counter(ds, -1, stream);
  const int use_k = prm->momentum ? 1 : 0;
  for (int k = 0; k < prm->iters; ++k) {
    if (k % U.ck == 0) {
      float2 *slot = ck + (size_t)(1 + 2 * (k / U.ck)) * n;
      PF_HIP(hipMemcpyAsync(slot, x, n * sizeof(float2), hipMemcpyDeviceToDevice, stream));
      PF_HIP(hipMemcpyAsync(slot + n, z, n * sizeof(float2), hipMemcpyDeviceToDevice, stream));
    }
    unroll_step(p, sens, mask, c, il, (float)prm->lambda, use_k, a, x, z, at<float2>(ws, U.base.img[1]),
                at<float2>(ws, U.base.img[2]), ws, stream, cand);
  }
  PF_HIP(hipMemcpyAsync(x_out, x, n * sizeof(float2), hipMemcpyDeviceToDevice, stream));
  return launch_status("pfista_unroll_forward");
}

int pfista_unroll_backward(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                           const pfista_unroll_params *prm, const pfista_c32 *x_bar, const void *ckpt, double *grad,
                           void *ws, hipStream_t stream) {
  PF_TRY(check_ops(p, sens, mask, ws));
  if (p->d.mask_kind == PFISTA_TOEPLITZ) return fail(PFISTA_UNSUPPORTED, "pfista_unroll_backward: Cartesian plans only");
  std::vector<double> c;
  PF_TRY(check_unroll(prm, c));
  if (!grad) return fail(PFISTA_EINVAL, "grad is NULL");
  const int deg = (int)c.size() - 1;
  for (int i = 0; i < deg + 2; ++i) grad[i] = 0.0;
  if (p->d.slices == 0) return PFISTA_OK;
  PF_TRY(check_ptr(x_bar, "x_bar"));
  PF_TRY(check_ptr(ckpt, "ckpt", 16));
  pfista_unroll_params q = *prm;
  q.degree = deg;
  q.coef = c.data();
  const ULayout U = ulayout(p->d, &q);
  const size_t n = U.base.n_img;
  if (n == 0) return PFISTA_OK;
  const pfista_desc &d = p->d;
  DevState *ds = at<DevState>(ws, U.base.state);
  double *partials = at<double>(ws, U.base.partials);
  const float2 *ck = static_cast<const float2 *>(ckpt);
  const float2 *a = ck;
  float2 *x = at<float2>(ws, U.x), *z = at<float2>(ws, U.z);
  float2 *seg = at<float2>(ws, U.seg);
  float2 *qb = at<float2>(ws, U.q), *pv = at<float2>(ws, U.pv);
  float2 *xb = at<float2>(ws, U.xb), *zb = at<float2>(ws, U.zb), *zb2 = at<float2>(ws, U.zb2);
  double *gdev = at<double>(ws, U.grad), *cpart = at<double>(ws, U.cpart);
  const double il = prm->inv_l;
  const float lam = (float)prm->lambda;
  const int use_k = prm->momentum ? 1 : 0;
  int cand = 0;
  PF_TRY(unroll_candidate(p, sens, mask, c, il, prm->tune, a, at<float2>(ws, U.base.img[1]),
                          at<float2>(ws, U.base.img[2]), ws, stream, cand));
  PF_HIP(hipMemsetAsync(gdev, 0, (size_t)(deg + 2) * sizeof(double), stream));
  PF_HIP(hipMemcpyAsync(xb, x_bar, n * sizeof(float2), hipMemcpyDeviceToDevice, stream));
  pf::k_fill<<<blocks_for(n), 256, 0, stream>>>(zb, n, make_float2(0.f, 0.f));
  pf::CoefArg carg{};
  for (int i = 0; i <= deg && i < 9; ++i) carg.c[i] = (float)c[i];
  float alpha[kMaxDegree + 1], beta0[kMaxDegree + 1];
  const float2 *wnull[kMaxDegree + 1];
  float2 *qy[kMaxDegree + 1];
  for (int i = 0; i < deg; ++i) {
    alpha[i] = (float)il;
    beta0[i] = 0.f;
    wnull[i] = nullptr;
    qy[i] = qb + (size_t)(i + 1) * n;
  }
  const dim3 sgrid(d.n / 16, d.n / 16, d.slices);
  const int nsb = (d.n / 16) * (d.n / 16) * d.slices;
  for (int j = U.nck - 1; j >= 0; --j) {
    const int k0 = j * U.ck, k1 = std::min(k0 + U.ck, prm->iters);
    // recompute the segment from its checkpoint, keeping z_k, g_k, pg_k
    PF_HIP(hipMemcpyAsync(x, ck + (size_t)(1 + 2 * j) * n, n * sizeof(float2), hipMemcpyDeviceToDevice, stream));
    PF_HIP(hipMemcpyAsync(z, ck + (size_t)(2 + 2 * j) * n, n * sizeof(float2), hipMemcpyDeviceToDevice, stream));
    set_counter(ds, k0 - 1, stream);
    for (int k = k0; k < k1; ++k) {
      float2 *sz = seg + (size_t)(3 * (k - k0)) * n;
      PF_HIP(hipMemcpyAsync(sz, z, n * sizeof(float2), hipMemcpyDeviceToDevice, stream));
      unroll_step(p, sens, mask, c, il, lam, use_k, a, x, z, sz + n, sz + 2 * n, ws, stream, cand);
    }
    // pull back through the segment's steps in reverse order
    for (int k = k1 - 1; k >= k0; --k) {
      const float2 *sz = seg + (size_t)(3 * (k - k0)) * n;
      const float beta = prm->momentum ? (float)((double)k / ((double)k + 3.0)) : 0.f;
      switch (d.haar_levels) {
        case 1: pf::k_prox_vjp<1><<<sgrid, 64, 0, stream>>>(sz, sz + 2 * n, xb, zb, qb, lam, beta, d.n, partials); break;
        case 2: pf::k_prox_vjp<2><<<sgrid, 64, 0, stream>>>(sz, sz + 2 * n, xb, zb, qb, lam, beta, d.n, partials); break;
        case 3: pf::k_prox_vjp<3><<<sgrid, 64, 0, stream>>>(sz, sz + 2 * n, xb, zb, qb, lam, beta, d.n, partials); break;
        default: pf::k_prox_vjp<4><<<sgrid, 64, 0, stream>>>(sz, sz + 2 * n, xb, zb, qb, lam, beta, d.n, partials); break;
      }
      pf::k_reduce_add<<<1, 64, 0, stream>>>(partials, nsb, 1, 1.0, gdev);
      if (deg > 0)
        chain_shaped(d, cand, sens, mask, qb, deg, alpha, beta0, wnull, qy, at<float2>(ws, U.base.t), stream,
                     nullptr);
      pf::k_poly_combine_dot<<<U.ncomb, 256, 0, stream>>>(qb, deg + 1, n, sz + n, carg, pv, cpart);
      pf::k_reduce_add<<<1, 64, 0, stream>>>(cpart, U.ncomb, deg + 1, -1.0, gdev + 1);
      // z_bar_k = v_bar - N' p(N') v_bar
      normal_op(d, sens, mask, pv, zb2, (float)(-il), qb, 1.f, ws, stream);
      std::swap(zb, zb2);
    }
    PF_TRY(launch_status("pfista_unroll_backward"));
  }
  PF_HIP(hipMemcpyAsync(grad, gdev, (size_t)(deg + 2) * sizeof(double), hipMemcpyDeviceToHost, stream));
  PF_HIP(hipStreamSynchronize(stream));
  return PFISTA_OK;
}

}  // extern "C"

// ============================================================================ non-Cartesian set-up
namespace {

int check_traj(const pfista_plan *p, const float *traj, int J) {
  PF_TRY(check_plan(p));
  if (p->d.mask_kind != PFISTA_TOEPLITZ) return fail(PFISTA_EINVAL, "plan is not a Toeplitz plan");
  if (J < 1) return fail(PFISTA_EINVAL, "J must be >= 1");
  if ((long long)J * p->d.slices * p->d.coils > (1ll << 31) - 1) return fail(PFISTA_UNSUPPORTED, "too many samples");
  return check_ptr(traj, "traj", 4);
}

unsigned grid_for(size_t n) { return (unsigned)std::max<size_t>(1, (n + 255) / 256); }

}  // namespace

extern "C" {

int pfista_toeplitz_kernel(const pfista_plan *p, const float *traj, const float *weights, int J, float *kern,
                           hipStream_t stream) {
  PF_TRY(check_traj(p, traj, J));
  if (weights) PF_TRY(check_ptr(weights, "weights", 4));
  PF_TRY(check_ptr(kern, "kern", 4));
  PF_TRY(ensure_twiddles());
  const size_t total = (size_t)p->d.slices * 4 * p->d.n * p->d.n;
  if (total == 0) return PFISTA_OK;
  pf::k_toeplitz_kernel<<<grid_for(total), 256, 0, stream>>>(traj, weights, J, p->d.n, p->d.slices, kern);
  return launch_status("pfista_toeplitz_kernel");
}

int pfista_nudft_forward(const pfista_plan *p, const pfista_c32 *sens, const float *traj, int J,
                         const pfista_c32 *x, pfista_c32 *kdata, hipStream_t stream) {
  PF_TRY(check_traj(p, traj, J));
  PF_TRY(check_ptr(sens, "sens"));
  PF_TRY(check_ptr(x, "x"));
  PF_TRY(check_ptr(kdata, "kdata"));
  const size_t total = (size_t)p->d.slices * p->d.coils * J;
  if (total == 0) return PFISTA_OK;
  pf::k_nudft_forward<<<grid_for(total), 256, 0, stream>>>(F2(sens), F2(x), traj, J, p->d.n, p->d.coils,
                                                           p->d.slices, F2(kdata));
  return launch_status("pfista_nudft_forward");
}

int pfista_nudft_adjoint(const pfista_plan *p, const pfista_c32 *sens, const float *traj, int J,
                         const pfista_c32 *kdata, pfista_c32 *y, hipStream_t stream) {
  PF_TRY(check_traj(p, traj, J));
  PF_TRY(check_ptr(sens, "sens"));
  PF_TRY(check_ptr(kdata, "kdata"));
  PF_TRY(check_ptr(y, "y"));
  const size_t total = (size_t)p->d.slices * p->d.n * p->d.n;
  if (total == 0) return PFISTA_OK;
  pf::k_nudft_adjoint<<<grid_for(total), 256, 0, stream>>>(F2(sens), F2(kdata), traj, J, p->d.n, p->d.coils,
                                                           p->d.slices, F2(y));
  return launch_status("pfista_nudft_adjoint");
}

}  // extern "C"
