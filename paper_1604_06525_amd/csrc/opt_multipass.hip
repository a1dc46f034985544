// Multi-pass optimisation (Sec. 7): the steps between solves, and the
// hierarchical (coarse-to-fine) optical flow of Appendix A.2.3 built from them.
//
// Between passes the problem state changes: images are resampled to the next
// level of a pyramid, the derivative images the flow energy samples (Sec. 7,
// sampled images) are recomputed for that level, and the coarse solution is
// carried to the finer grid as its starting point.  Each step is one kernel
// over the sites of a level; a level's solve is an ordinary opt_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "opt.h"
#include "host.h"

using namespace optmi;
using namespace optmi::host;

namespace {

constexpr int kMaxPlanes = 8;

// dst (floor(W/2) x floor(H/2) per plane) = mean of each 2 x 2 block of src.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_downsample2(const T* __restrict__ src, int W, int H, int planes,
                                                        T* __restrict__ dst) {
  const int Wd = W / 2, Hd = H / 2;
  const long long n = (long long)Wd * Hd, total = n * planes;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total; t += (long long)gridDim.x * kBlock) {
    const int c = (int)(t / n);
    const long long s = t - (long long)c * n;
    const int i = (int)(s % Wd), j = (int)(s / Wd);
    const T* p = src + (size_t)c * W * H + (size_t)(2 * j) * W + 2 * i;
    dst[t] = T(0.25) * ((p[0] + p[1]) + (p[W] + p[W + 1]));
  }
}

// Derivative images along the width (dx) and the height (dy): central
// differences inside, one-sided differences on the first and last column
// (row), 0 along a dimension of one sample.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gradient(const T* __restrict__ img, int W, int H, T* __restrict__ dx,
                                                     T* __restrict__ dy) {
  const long long n = (long long)W * H;
  for (long long s = (long long)blockIdx.x * kBlock + threadIdx.x; s < n; s += (long long)gridDim.x * kBlock) {
    const int i = (int)(s % W), j = (int)(s / W);
    T gx = T(0), gy = T(0);
    if (W > 1) {
      if (i == 0) gx = img[s + 1] - img[s];
      else if (i == W - 1) gx = img[s] - img[s - 1];
      else gx = (img[s + 1] - img[s - 1]) * T(0.5);
    }
    if (H > 1) {
      if (j == 0) gy = img[s + W] - img[s];
      else if (j == H - 1) gy = img[s] - img[s - W];
      else gy = (img[s + W] - img[s - W]) * T(0.5);
    }
    dx[s] = gx;
    dy[s] = gy;
  }
}

template <typename T>
struct Scales {
  T v[kMaxPlanes];
};

// Value of a plane's scale (a select, not an index into the argument struct).
template <typename T>
__device__ __forceinline__ T pick_plane(const Scales<T>& s, int c) {
  T v = s.v[0];
#pragma unroll
  for (int k = 1; k < kMaxPlanes; ++k) v = c == k ? s.v[k] : v;
  return v;
}

// dst(i, j) of plane c = scale_c * S(src_c; x, y) with x = (i + 1/2) Ws/Wd - 1/2,
// y = (j + 1/2) Hs/Hd - 1/2: the bilinear, clamp-to-edge sample (texel centres
// at integer coordinates) at the point of the coarse grid that covers the fine
// pixel's centre.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_upsample(const T* __restrict__ src, int Ws, int Hs, int planes,
                                                     Scales<T> sc, T* __restrict__ dst, int Wd, int Hd) {
  const long long n = (long long)Wd * Hd, total = n * planes;
  const T rx = T(Ws) / T(Wd), ry = T(Hs) / T(Hd);
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total; t += (long long)gridDim.x * kBlock) {
    const int c = (int)(t / n);
    const long long s = t - (long long)c * n;
    const int i = (int)(s % Wd), j = (int)(s / Wd);
    const T x = (T(i) + T(0.5)) * rx - T(0.5), y = (T(j) + T(0.5)) * ry - T(0.5);
    const T x0 = floor(x), y0 = floor(y);
    const T fx = x - x0, fy = y - y0;
    const int ix0 = min(max((int)x0, 0), Ws - 1), ix1 = min(max((int)x0 + 1, 0), Ws - 1);
    const int iy0 = min(max((int)y0, 0), Hs - 1), iy1 = min(max((int)y0 + 1, 0), Hs - 1);
    const T* p = src + (size_t)c * Ws * Hs;
    const T v = (T(1) - fx) * (T(1) - fy) * p[(size_t)iy0 * Ws + ix0] + fx * (T(1) - fy) * p[(size_t)iy0 * Ws + ix1] +
                (T(1) - fx) * fy * p[(size_t)iy1 * Ws + ix0] + fx * fy * p[(size_t)iy1 * Ws + ix1];
    dst[t] = pick_plane(sc, c) * v;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_zero(T* __restrict__ dst, long long n) {
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < n; t += (long long)gridDim.x * kBlock)
    dst[t] = T(0);
}

int grid_for(long long work) {
  return (int)std::max<long long>(1, std::min<long long>(8 * 1024, (work + kBlock - 1) / kBlock));
}

int check_precision(int32_t precision) {
  if (precision != OPT_FP64 && precision != OPT_MIXED)
    return fail(OPT_EINVAL, "precision %d is not OPT_FP64 or OPT_MIXED", precision);
  return OPT_OK;
}

template <typename T>
int downsample_t(const void* src, int W, int H, int planes, void* dst, hipStream_t st) {
  const long long work = (long long)(W / 2) * (H / 2) * planes;
  k_downsample2<T><<<grid_for(work), kBlock, 0, st>>>((const T*)src, W, H, planes, (T*)dst);
  HIP_LAUNCHED("downsample2");
  return OPT_OK;
}

template <typename T>
int gradient_t(const void* img, int W, int H, void* dx, void* dy, hipStream_t st) {
  k_gradient<T><<<grid_for((long long)W * H), kBlock, 0, st>>>((const T*)img, W, H, (T*)dx, (T*)dy);
  HIP_LAUNCHED("gradient");
  return OPT_OK;
}

template <typename T>
int upsample_t(const void* src, int Ws, int Hs, int planes, const double* scale, void* dst, int Wd, int Hd,
               hipStream_t st) {
  Scales<T> sc{};
  for (int c = 0; c < planes; ++c) sc.v[c] = (T)scale[c];
  k_upsample<T><<<grid_for((long long)Wd * Hd * planes), kBlock, 0, st>>>((const T*)src, Ws, Hs, planes, sc,
                                                                           (T*)dst, Wd, Hd);
  HIP_LAUNCHED("upsample");
  return OPT_OK;
}

template <typename T>
int zero_t(void* dst, long long n, hipStream_t st) {
  k_zero<T><<<grid_for(n), kBlock, 0, st>>>((T*)dst, n);
  HIP_LAUNCHED("zero");
  return OPT_OK;
}

// ---------------------------------------------------------------- flow pyramid
// Level l of a pyramid of `levels` has floor(W / 2^l) x floor(H / 2^l) pixels;
// the coarsest must keep at least kMinSide on each side.
constexpr int kMinSide = 4;

struct PyramidLayout {
  int levels = 0;
  std::vector<int> W, H;
  std::vector<size_t> I, Ih, dx, dy, x;  // byte offsets (level 0 images are the caller's)
  size_t prob = 0, prob_bytes = 0, total = 0;
};

opt_problem_desc flow_desc(int W, int H, int precision, const void* I, const void* Ih, const void* dx,
                           const void* dy, double w_fit, double w_reg) {
  opt_problem_desc d{};
  d.domain = OPT_GRID2D;
  d.energy = OPT_E_FLOW;
  d.precision = precision;
  d.width = W;
  d.height = H;
  d.arrays[0] = I;
  d.arrays[1] = Ih;
  d.arrays[2] = dx;
  d.arrays[3] = dy;
  d.params[0] = w_fit;
  d.params[1] = w_reg;
  d.n_params = 2;
  return d;
}

int pyramid_layout(int W, int H, int levels, int precision, PyramidLayout* L) {
  TRY(check_precision(precision));
  if (W < 1 || H < 1) return fail(OPT_EINVAL, "grid size %d x %d must be positive", W, H);
  if (levels < 1 || levels > 16) return fail(OPT_EINVAL, "levels %d outside [1, 16]", levels);
  if ((W >> (levels - 1)) < kMinSide || (H >> (levels - 1)) < kMinSide)
    return fail(OPT_EINVAL, "%d levels of a %d x %d grid leave a coarsest level under %d x %d", levels, W, H,
                kMinSide, kMinSide);
  const size_t ts = precision == OPT_FP64 ? sizeof(double) : sizeof(float);
  L->levels = levels;
  L->W.assign(levels, 0);
  L->H.assign(levels, 0);
  L->I.assign(levels, 0);
  L->Ih.assign(levels, 0);
  L->dx.assign(levels, 0);
  L->dy.assign(levels, 0);
  L->x.assign(levels, 0);
  size_t off = 0;
  for (int l = 0; l < levels; ++l) {
    L->W[l] = W >> l;
    L->H[l] = H >> l;
    const size_t plane = align_up((size_t)L->W[l] * L->H[l] * ts);
    if (l > 0) {
      L->I[l] = off;
      off += plane;
      L->Ih[l] = off;
      off += plane;
      L->x[l] = off;
      off += 2 * plane;
    }
    L->dx[l] = off;
    off += plane;
    L->dy[l] = off;
    off += plane;
    // the problem workspace of this level (shared by all levels)
    const int dummy = 1;
    opt_problem_desc d = flow_desc(L->W[l], L->H[l], precision, &dummy, &dummy, &dummy, &dummy, 1.0, 1.0);
    Shape sh;
    TRY(check_desc(&d, &sh));
    L->prob_bytes = std::max(L->prob_bytes, align_up(make_layout(sh).total));
  }
  L->prob = off;
  L->total = off + L->prob_bytes;
  return OPT_OK;
}

template <typename T>
int solve_pyramid_t(const void* I, const void* Ih, int levels, double w_fit, double w_reg, int precision,
                    const opt_solve_params* sp, void* unknowns, char* ws, const PyramidLayout& L, hipStream_t st,
                    opt_solve_report* reports) {
  auto img = [&](int l) -> const void* { return l == 0 ? I : (const void*)(ws + L.I[l]); };
  auto himg = [&](int l) -> const void* { return l == 0 ? Ih : (const void*)(ws + L.Ih[l]); };
  auto xof = [&](int l) -> void* { return l == 0 ? unknowns : (void*)(ws + L.x[l]); };
  // the image pyramid, then the derivative images of every level
  for (int l = 1; l < levels; ++l) {
    TRY(downsample_t<T>(img(l - 1), L.W[l - 1], L.H[l - 1], 1, ws + L.I[l], st));
    TRY(downsample_t<T>(himg(l - 1), L.W[l - 1], L.H[l - 1], 1, ws + L.Ih[l], st));
  }
  for (int l = 0; l < levels; ++l) TRY(gradient_t<T>(himg(l), L.W[l], L.H[l], ws + L.dx[l], ws + L.dy[l], st));
  // coarse to fine: the coarsest level starts from zero flow; each finer level
  // from the solution of the level below, resampled and scaled to its pixels
  if (levels > 1) TRY(zero_t<T>(xof(levels - 1), 2LL * L.W[levels - 1] * L.H[levels - 1], st));
  for (int l = levels - 1; l >= 0; --l) {
    const opt_problem_desc d =
        flow_desc(L.W[l], L.H[l], precision, img(l), himg(l), ws + L.dx[l], ws + L.dy[l], w_fit, w_reg);
    Shape sh;
    TRY(check_desc(&d, &sh));
    opt_problem p;
    TRY(problem_init(&p, &d, sh, ws + L.prob, st));
    TRY(solve(&p, xof(l), sp, reports ? &reports[l] : nullptr));
    if (l > 0) {
      const double scale[2] = {(double)L.W[l - 1] / L.W[l], (double)L.H[l - 1] / L.H[l]};
      TRY(upsample_t<T>(xof(l), L.W[l], L.H[l], 2, scale, xof(l - 1), L.W[l - 1], L.H[l - 1], st));
    }
  }
  return OPT_OK;
}

}  // namespace

extern "C" {

int opt_image_downsample2(const void* src, int32_t width, int32_t height, int32_t planes, int32_t precision,
                          void* dst, void* hip_stream) {
  TRY(check_precision(precision));
  if (!src || !dst) return fail(OPT_EINVAL, "src or dst is NULL");
  if (width < 2 || height < 2) return fail(OPT_EINVAL, "grid %d x %d is too small to halve", width, height);
  if (planes < 1 || planes > kMaxPlanes) return fail(OPT_EINVAL, "planes %d outside [1, %d]", planes, kMaxPlanes);
  hipStream_t st = (hipStream_t)hip_stream;
  return precision == OPT_FP64 ? downsample_t<double>(src, width, height, planes, dst, st)
                               : downsample_t<float>(src, width, height, planes, dst, st);
}

int opt_image_gradient(const void* img, int32_t width, int32_t height, int32_t precision, void* dx, void* dy,
                       void* hip_stream) {
  TRY(check_precision(precision));
  if (!img || !dx || !dy) return fail(OPT_EINVAL, "img, dx or dy is NULL");
  if (width < 1 || height < 1) return fail(OPT_EINVAL, "grid size %d x %d must be positive", width, height);
  hipStream_t st = (hipStream_t)hip_stream;
  return precision == OPT_FP64 ? gradient_t<double>(img, width, height, dx, dy, st)
                               : gradient_t<float>(img, width, height, dx, dy, st);
}

int opt_field_upsample(const void* src, int32_t src_width, int32_t src_height, int32_t planes,
                       const double* scale, int32_t precision, void* dst, int32_t dst_width, int32_t dst_height,
                       void* hip_stream) {
  TRY(check_precision(precision));
  if (!src || !dst || !scale) return fail(OPT_EINVAL, "src, dst or scale is NULL");
  if (src_width < 1 || src_height < 1 || dst_width < 1 || dst_height < 1)
    return fail(OPT_EINVAL, "grid sizes must be positive");
  if (planes < 1 || planes > kMaxPlanes) return fail(OPT_EINVAL, "planes %d outside [1, %d]", planes, kMaxPlanes);
  hipStream_t st = (hipStream_t)hip_stream;
  return precision == OPT_FP64
             ? upsample_t<double>(src, src_width, src_height, planes, scale, dst, dst_width, dst_height, st)
             : upsample_t<float>(src, src_width, src_height, planes, scale, dst, dst_width, dst_height, st);
}

int opt_flow_pyramid_workspace_size(int32_t width, int32_t height, int32_t levels, int32_t precision,
                                    size_t* bytes) {
  if (!bytes) return fail(OPT_EINVAL, "bytes is NULL");
  PyramidLayout L;
  TRY(pyramid_layout(width, height, levels, precision, &L));
  *bytes = L.total;
  return OPT_OK;
}

int opt_solve_flow_pyramid(const void* I, const void* I_hat, int32_t width, int32_t height, int32_t levels,
                           double w_fit, double w_reg, int32_t precision, const opt_solve_params* params,
                           void* unknowns, void* workspace, size_t workspace_bytes, void* hip_stream,
                           opt_solve_report* reports) {
  if (!I || !I_hat || !unknowns || !workspace) return fail(OPT_EINVAL, "I, I_hat, unknowns or workspace is NULL");
  PyramidLayout L;
  TRY(pyramid_layout(width, height, levels, precision, &L));
  TRY(check_params(params));
  if (((uintptr_t)workspace) % kAlign) return fail(OPT_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < L.total)
    return fail(OPT_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, L.total);
  hipStream_t st = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  return precision == OPT_FP64
             ? solve_pyramid_t<double>(I, I_hat, levels, w_fit, w_reg, precision, params, unknowns, ws, L, st,
                                       reports)
             : solve_pyramid_t<float>(I, I_hat, levels, w_fit, w_reg, precision, params, unknowns, ws, L, st,
                                      reports);
}

}  // extern "C"
