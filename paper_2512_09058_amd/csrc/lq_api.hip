// Host runtime of liblqkkt: plans, argument validation, workspace layout, kernel dispatch.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "lq_internal.hpp"
#include "lq_qp.hpp"
#include "lqpit.h"
#include "lqupdate.h"

namespace lq {
size_t generic_factor_lds(int nx, int nu);
size_t generic_solve_lds(int nx, int nu);
size_t generic_stage_doubles(int nx, int nu);
hipError_t launch_factor_generic(lq_mode mode, const Desc* desc, int batch, const lq_data& d, void* F,
                                 double* V, int32_t* info, size_t lds, const GenericLaunch& c, hipStream_t st);
hipError_t launch_solve_generic(lq_mode mode, const SolveArgs& a, size_t lds, const GenericLaunch& c,
                                hipStream_t st);
hipError_t prepare_generic(bool factor, size_t lds);
int generic_blocks_per_cu(int threads, size_t lds, bool factor, lq_mode mode);
hipError_t launch_grad_generic(const GradArgs& a, hipStream_t st);

// Size-specialised uniform-batch kernels (lq_small.hip); return false if no variant fits.
bool small_variant_available(lq_mode mode, int nx, int nu);
bool small_aligned(const lq_data& d, const void* ws);
hipError_t launch_factor_small(lq_mode mode, int batch, int N, int nx, int nu, const lq_data& d,
                               void* F, double* V, int32_t* info, hipStream_t st);
hipError_t launch_solve_small(lq_mode mode, int N, int nx, int nu, const SolveArgs& a, hipStream_t st);
// Smallest compiled size-specialised shape covering (nx, nu) (lq_small.hip).
bool small_envelope(lq_mode mode, int nx, int nu, int* NX, int* NU);
// Copies to and from a padded problem, real factor blocks from padded ones (lq_pad.hip).
hipError_t launch_pad(const PadOp* ops, int n, hipStream_t st);
hipError_t launch_extract_small_factors(bool f64, const void* src, void* dst, int64_t blocks, int nx, int nu, int NX,
                                        int NU, hipStream_t st);

// Matrix-core tile factor kernels (lq_tile.hip).
int tile_max_columns();
int tile_waves(int T);
bool tile_mode_supported(lq_mode mode);
size_t tile_lds_bytes(int nx, int nu, lq_mode mode);
hipError_t prepare_tile(int waves, lq_mode mode, size_t lds);
int tile_blocks_per_cu(int waves, lq_mode mode, size_t lds);
hipError_t launch_factor_tile(lq_mode mode, int waves, const Desc* desc, int batch, const lq_data& d, void* F,
                              double* V, int32_t* info, size_t lds, const GenericLaunch& c, hipStream_t st);

// Register-streaming solve kernels for nx <= 128, nu <= 64 (lq_tsolve.hip).
bool tsolve_sizes(int maxnx, int maxnu, int* NXP, int* NUP);
size_t tsolve_lds_bytes(int NXP, int NUP);
hipError_t prepare_tsolve(int NXP, int NUP, lq_mode mode);
int tsolve_blocks_per_cu(int NXP, int NUP, lq_mode mode);
hipError_t launch_solve_tsolve(int NXP, int NUP, lq_mode mode, const SolveArgs& a, const GenericLaunch& c,
                               hipStream_t st);

// Checkpointed solve kernels of tile plans, nx <= 64 with nu <= 64 or nx <= 128 with nu <= 32 (lq_tckpt.hip).
bool tckpt_sizes(int maxnx, int maxnu, int* NXP, int* NUP);
bool tckpt_mode_supported(lq_mode mode);
int tckpt_waves(int NXP, int NUP);
size_t tckpt_lds_bytes(int NXP, int NUP, size_t tile_lds);
hipError_t prepare_tckpt(int NXP, int NUP, lq_mode mode, size_t lds);
int tckpt_blocks_per_cu(int NXP, int NUP, lq_mode mode, size_t lds);
hipError_t launch_solve_tckpt(int NXP, int NUP, lq_mode mode, const SolveArgs& a, size_t lds,
                              const GenericLaunch& c, hipStream_t st);
// lq_update.hip
int update_width(int lrsmax, int lqmax, int nuxmax, int nxmax, int* ldy_out);
bool update_sweep_fits(int fsmax, int nuxmax, int nxmax);
void update_ws_layout(int wmax, int64_t sum_Nnx, int64_t sum_K, int batch, size_t* oSg, size_t* oWk, size_t* oSt,
                      size_t* total);
hipError_t launch_update_data(const Desc* desc, int batch, int maxN, const lq_update& u, double* Q, double* R,
                              double* S, hipStream_t st);
hipError_t launch_factor_update(const Desc* desc, int batch, int maxN, int lrsmax, int lqmax, int fsmax, int nuxmax,
                                int nxmax, int64_t sum_Nnx, int64_t sum_K, const lq_data& d, const lq_update& u,
                                double* F, double* V, void* uws, int32_t* info, hipStream_t st);
}  // namespace lq

namespace lq {
// Raise (never lower) a kernel's dynamic-LDS limit: plans of different sizes share the kernels, and
// a later plan must not lower the limit an earlier one launches with.
hipError_t raise_lds_limit(const void* kernel, size_t lds) {
  static std::mutex mu;
  static std::map<const void*, size_t> set;
  std::lock_guard<std::mutex> lock(mu);
  auto it = set.find(kernel);
  if (it != set.end() && it->second >= lds) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) set[kernel] = lds;
  return e;
}
}  // namespace lq

using lq::Desc;

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace lq {
int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
void clear_error() { g_err.clear(); }
}  // namespace lq

static const size_t kLdsLimit = 160 * 1024;

enum Variant : int32_t { VAR_GENERIC = 0, VAR_SMALL = 1, VAR_TILE = 2, VAR_SMALL_PAD = 3 };

struct lq_plan {
  int32_t batch = 0;
  lq_mode mode = LQ_F64;
  int32_t ckpt = 0;
  bool uniform = true;
  int32_t maxN = 0, maxnx = 0, maxnu = 0;
  std::vector<int32_t> N, nx, nu;
  std::vector<int64_t> off[LQ_ARR_COUNT];
  int64_t total[LQ_ARR_COUNT] = {};
  std::vector<Desc> desc_h;
  Desc* desc_d = nullptr;
  int device = 0;
  size_t fbytes = 0;  // bytes per factor element
  size_t offF = 0, offV = 0, offV2 = 0, offZB = 0, ws_bytes = 0;
  size_t lds_factor = 0, lds_solve = 0;
  size_t stage_doubles = 0;  // staging buffer of the solve kernels
  Variant variant = VAR_GENERIC;
  bool can_small = false, can_tile = false, can_generic = false;
  int tile_waves = 0;       // wavefronts per workgroup of the tile factor kernel
  size_t lds_tile = 0;      // its dynamic LDS bytes
  int ts_nxp = 0, ts_nup = 0;  // padded sizes of the tile plan's solve kernel (0: generic solve)
  size_t lds_tckpt = 0;        // checkpointed tile plans: LDS of the solve kernel
  int32_t* order_d = nullptr;  // device: instance indices longest first (inside the desc allocation)
  // Ragged tile plans: instances grouped by kernel shape (factor wavefronts, padded solve sizes),
  // one launch per group, heaviest group first (empty: one launch for the whole batch).
  struct Bucket {
    int waves, nxp, nup;
    int32_t off, cnt;          // positions [off, off + cnt) of border_d
    size_t lds_tile;
    int32_t grid_factor, grid_solve;
  };
  std::vector<Bucket> buckets;
  int32_t* border_d = nullptr;  // device: instance indices grouped by bucket, longest first within
  // Streams on which the groups after the first run beside it, forked from and joined back into
  // the caller's stream with events (capturable into a graph): ev[0] marks the fork, ev[i] the end
  // of group i.  Empty when the plan launches one group (or could not create them: the groups then
  // run one after another on the caller's stream).
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
  size_t offCtr = 0;           // workspace: work counters of the persistent kernels
  int cu_count = 0;
  lq_launch launch = {128, 0, 0, 0};
  int32_t grid_factor = 0, grid_solve = 0;  // persistent grid sizes for `launch`
  // Uniform plans whose shape has no size-specialised kernel but fits in a compiled one
  // (VAR_SMALL_PAD): the plan of that padded shape, whose workspace follows this plan's regions at
  // offPad, then the padded data and outputs (A, B, Q, R, S, q, r, f, x0, x, u, lam).
  bool can_small_pad = false;
  int pad_nx = 0, pad_nu = 0;
  lq_plan* inner = nullptr;
  size_t offPad = 0;
  size_t offPadArr[12] = {};
  ~lq_plan() { lq_plan_destroy(inner); }
};

// Persistent grid sizes for the plan's launch shape (host queries; done outside the calls so
// that lq_factor / lq_solve only enqueue kernels and stay capturable in a graph).
static void update_grids(lq_plan* p) {
  for (auto& b : p->buckets) {
    int pf = lq::tile_blocks_per_cu(b.waves, p->mode, b.lds_tile);
    int ps = lq::tsolve_blocks_per_cu(b.nxp, b.nup, p->mode);
    if (p->launch.blocks_per_cu > 0) {
      pf = std::min(pf, (int)p->launch.blocks_per_cu);
      ps = std::min(ps, (int)p->launch.blocks_per_cu);
    }
    b.grid_factor = (int32_t)std::min((int64_t)p->cu_count * pf, (int64_t)b.cnt);
    b.grid_solve = (int32_t)std::min((int64_t)p->cu_count * ps, (int64_t)b.cnt);
  }
  for (int f = 0; f < 2; ++f) {
    const size_t lds = f ? p->lds_factor : p->lds_solve;
    int per;
    if (p->variant == VAR_TILE)
      per = f ? lq::tile_blocks_per_cu(p->tile_waves, p->mode, p->lds_tile)
              : p->ckpt ? lq::tckpt_blocks_per_cu(p->ts_nxp, p->ts_nup, p->mode, p->lds_tckpt)
              : p->ts_nxp ? lq::tsolve_blocks_per_cu(p->ts_nxp, p->ts_nup, p->mode)
                          : lq::generic_blocks_per_cu(p->launch.threads, lds, false, p->mode);
    else
      per = lq::generic_blocks_per_cu(p->launch.threads, lds, f != 0, p->mode);
    if (p->launch.blocks_per_cu > 0 && p->launch.blocks_per_cu < per) per = p->launch.blocks_per_cu;
    const int64_t g = (int64_t)p->cu_count * per;
    const int32_t grid = (int32_t)(g < p->batch ? g : p->batch);
    (f ? p->grid_factor : p->grid_solve) = grid;
  }
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

extern "C" int lq_version(void) { return 100; }

extern "C" const char* lq_last_error(void) { return g_err.c_str(); }

extern "C" int lq_plan_create(int32_t batch, const int32_t* N, const int32_t* nx, const int32_t* nu,
                              lq_mode mode, int32_t ckpt_stride, lq_plan** out) {
  g_err.clear();
  if (!out) return fail(LQ_EINVAL, "lq_plan_create: out is NULL");
  *out = nullptr;
  if (batch <= 0) return fail(LQ_EINVAL, "lq_plan_create: batch must be positive (got %d)", batch);
  if (!N || !nx || !nu) return fail(LQ_EINVAL, "lq_plan_create: N, nx, nu host arrays are required");
  if (mode != LQ_F64 && mode != LQ_MIXED_F32 && mode != LQ_MIXED_BF16)
    return fail(LQ_EINVAL, "lq_plan_create: unknown mode %d", (int)mode);
  if (ckpt_stride < 0) return fail(LQ_EINVAL, "lq_plan_create: ckpt_stride must be >= 0");
  lq_plan* p = new (std::nothrow) lq_plan;
  if (!p) return fail(LQ_ENOMEM, "lq_plan_create: host allocation failed");
  p->batch = batch;
  p->mode = mode;
  p->ckpt = ckpt_stride;
  p->N.assign(N, N + batch);
  p->nx.assign(nx, nx + batch);
  p->nu.assign(nu, nu + batch);
  for (int i = 0; i < batch; ++i) {
    if (N[i] <= 0 || nx[i] <= 0 || nu[i] <= 0) {
      delete p;
      return fail(LQ_EINVAL, "lq_plan_create: instance %d has non-positive size (N=%d nx=%d nu=%d)", i,
                  N[i], nx[i], nu[i]);
    }
    if (N[i] > (1 << 24) || nx[i] > 4096 || nu[i] > 4096) {
      delete p;
      return fail(LQ_EUNSUPPORTED, "lq_plan_create: instance %d too large", i);
    }
    p->maxN = std::max(p->maxN, N[i]);
    p->maxnx = std::max(p->maxnx, nx[i]);
    p->maxnu = std::max(p->maxnu, nu[i]);
    if (N[i] != N[0] || nx[i] != nx[0] || nu[i] != nu[0]) p->uniform = false;
  }
  p->fbytes = mode == LQ_F64 ? sizeof(double) : sizeof(float);
  // packed layouts and per-instance descriptors
  for (int a = 0; a < LQ_ARR_COUNT; ++a) p->off[a].resize(batch);
  p->desc_h.resize(batch);
  int64_t acc[LQ_ARR_COUNT] = {};
  int64_t aF = 0, aV = 0, aV2 = 0, aZB = 0, aK = 0;
  size_t ldsf = 0, ldss = 0;
  for (int i = 0; i < batch; ++i) {
    const int64_t n = N[i], x = nx[i], u = nu[i];
    const int64_t sz[LQ_ARR_COUNT] = {n * x * x, n * x * u, (n + 1) * x * x, n * u * u, n * u * x,
                                      (n + 1) * x, n * u, n * x, x, n * x, n * u, n * x};
    for (int a = 0; a < LQ_ARR_COUNT; ++a) {
      p->off[a][i] = acc[a];
      acc[a] += sz[a];
    }
    Desc& D = p->desc_h[i];
    D.N = N[i]; D.nx = nx[i]; D.nu = nu[i]; D.pad = 0;
    D.oA = p->off[LQ_ARR_A][i]; D.oB = p->off[LQ_ARR_B][i]; D.oQ = p->off[LQ_ARR_Q][i];
    D.oR = p->off[LQ_ARR_R][i]; D.oS = p->off[LQ_ARR_S][i]; D.oq = p->off[LQ_ARR_q][i];
    D.or_ = p->off[LQ_ARR_r][i]; D.of = p->off[LQ_ARR_f][i]; D.ox0 = p->off[LQ_ARR_x0][i];
    D.ox = p->off[LQ_ARR_x][i]; D.ou = p->off[LQ_ARR_u][i]; D.olam = p->off[LQ_ARR_lam][i];
    D.oF = aF;
    if (ckpt_stride > 0) {
      // checkpoint slots (stages 0, s, 2s, ..., N) and one segment buffer of s stage blocks
      aF += (lq::ckpt_slots(n, ckpt_stride) + ckpt_stride) * lq::stage_factor_elems(nx[i], nu[i]);
    } else {
      aF += (n + 1) * lq::stage_factor_elems(nx[i], nu[i]);
    }
    D.oV = aV; aV += n * u + (n + 1) * x;
    D.oV2 = aV2; aV2 += lq::v2_elems(n, x, u);
    D.oZB = aZB; aZB += n * (2 * x + u);
    D.oK = aK; aK += n + 1;
    ldsf = std::max(ldsf, lq::generic_factor_lds(nx[i], nu[i]));
    ldss = std::max(ldss, lq::generic_solve_lds(nx[i], nu[i]));
    p->stage_doubles = std::max(p->stage_doubles, lq::generic_stage_doubles(nx[i], nu[i]));
  }
  ldss += sizeof(double) * p->stage_doubles;
  for (int a = 0; a < LQ_ARR_COUNT; ++a) p->total[a] = acc[a];
  p->lds_factor = ldsf;
  // a checkpointed solve recomputes factor segments: its LDS holds the factor scratch too
  p->lds_solve = ckpt_stride > 0 ? ldsf + ldss : ldss;
  // kernel variants that can take this batch; the first available of small, tile, generic is used
  int maxT = 0;
  for (int i = 0; i < batch; ++i) maxT = std::max(maxT, (nx[i] + 15) / 16 + (nu[i] + 15) / 16);
  p->can_small = p->uniform && ckpt_stride == 0 && lq::small_variant_available(mode, nx[0], nu[0]);
  p->can_generic = ldsf <= kLdsLimit && p->lds_solve <= kLdsLimit && mode != LQ_MIXED_BF16;
  if (lq::tile_mode_supported(mode) && maxT <= lq::tile_max_columns() && p->maxnu <= 64) {
    size_t lt = 0;
    for (int i = 0; i < batch; ++i) lt = std::max(lt, lq::tile_lds_bytes(nx[i], nu[i], mode));
    p->lds_tile = lt;
    if (ckpt_stride == 0) {
      p->tile_waves = lq::tile_waves(maxT);
      p->can_tile = lt <= kLdsLimit && p->lds_solve <= kLdsLimit;
    } else if (lq::tckpt_mode_supported(mode) && lq::tckpt_sizes(p->maxnx, p->maxnu, &p->ts_nxp, &p->ts_nup)) {
      // the solve recomputes segments with the factor sweep: both kernels use the same wavefront
      // count, so that the recomputed blocks are the factor kernel's bit for bit
      p->tile_waves = lq::tckpt_waves(p->ts_nxp, p->ts_nup);
      p->lds_tckpt = lq::tckpt_lds_bytes(p->ts_nxp, p->ts_nup, lt);
      p->can_tile = lt <= kLdsLimit && p->lds_tckpt <= kLdsLimit;
    }
  }
  p->variant = p->can_small ? VAR_SMALL : p->can_tile ? VAR_TILE : VAR_GENERIC;
  if (p->variant == VAR_GENERIC && !p->can_generic) {
    const size_t need = ldsf > p->lds_solve ? ldsf : p->lds_solve;
    delete p;
    if (mode == LQ_MIXED_BF16)
      return fail(LQ_EUNSUPPORTED, "lq_plan_create: LQ_MIXED_BF16 has no kernel for these sizes");
    return fail(LQ_EUNSUPPORTED, "lq_plan_create: stage tile needs %zu bytes of LDS (limit %zu)", need,
                kLdsLimit);
  }
  p->offF = 0;
  p->offV = align256(p->offF + (size_t)aF * p->fbytes);
  p->offV2 = align256(p->offV + (size_t)aV * sizeof(double));
  p->offZB = align256(p->offV2 + (size_t)aV2 * sizeof(double));
  p->offCtr = align256(p->offZB + (size_t)aZB * sizeof(double));
  p->ws_bytes = p->offCtr + 256;
  // a uniform shape without a size-specialised kernel of its own runs padded to the smallest
  // compiled shape that covers it (identity cost, no coupling on the padding; see lq_pad.hip)
  int env_nx = 0, env_nu = 0;
  // (32-bit row indices in the copy kernels: the padded arrays stay below 2^31 / 16 rows)
  if (p->uniform && ckpt_stride == 0 && !p->can_small && (int64_t)batch * (N[0] + 1) * 16 < ((int64_t)1 << 27) &&
      lq::small_envelope(mode, nx[0], nu[0], &env_nx, &env_nu)) {
    std::vector<int32_t> en(batch, env_nx), eu(batch, env_nu);
    lq_plan* in = nullptr;
    if (lq_plan_create(batch, N, en.data(), eu.data(), mode, 0, &in) == LQ_OK && in->variant == VAR_SMALL) {
      const int64_t b = batch, n = N[0], X = env_nx, U = env_nu;
      const int64_t elems[12] = {b * n * X * X, b * n * X * U, b * (n + 1) * X * X, b * n * U * U, b * n * U * X,
                                 b * (n + 1) * X, b * n * U, b * n * X, b * X, b * n * X, b * n * U, b * n * X};
      size_t o = align256(p->ws_bytes);
      p->offPad = o;
      o = align256(o + in->ws_bytes);
      for (int k = 0; k < 12; ++k) {
        p->offPadArr[k] = o;
        o = align256(o + (size_t)elems[k] * sizeof(double));
      }
      p->ws_bytes = o;
      p->inner = in;
      p->pad_nx = env_nx;
      p->pad_nu = env_nu;
      p->can_small_pad = true;
      p->variant = VAR_SMALL_PAD;
    } else {
      lq_plan_destroy(in);
    }
    g_err.clear();
  }
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(LQ_EHIP, "lq_plan_create: hipGetDevice failed");
  }
  if (hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
    (void)hipGetLastError();
    p->cu_count = 0;
  }
  if (p->cu_count <= 0) p->cu_count = 256;  // (only sizes persistent grids)
  // longest instances first: serial Riccati operation count of each instance
  std::vector<int32_t> order(batch);
  std::vector<double> cost(batch);
  for (int i = 0; i < batch; ++i) {
    const double x = nx[i], ux = nx[i] + nu[i];
    cost[i] = (double)N[i] * (0.5 * ux * x * x + 0.5 * ux * ux * x + ux * ux * ux / 6.0);
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t a_, int32_t b_) { return cost[a_] > cost[b_]; });
  const size_t descb = align256(sizeof(Desc) * batch);
  if (hipMalloc((void**)&p->desc_d, descb + 2 * sizeof(int32_t) * batch) != hipSuccess) {
    delete p;
    return fail(LQ_ENOMEM, "lq_plan_create: descriptor table allocation failed");
  }
  p->order_d = (int32_t*)((char*)p->desc_d + descb);
  p->border_d = p->order_d + batch;
  if (hipMemcpy(p->desc_d, p->desc_h.data(), sizeof(Desc) * batch, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->order_d, order.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->desc_d);  // cleanup of a failed creation
    delete p;
    return fail(LQ_EHIP, "lq_plan_create: descriptor upload failed");
  }
  // Raise the dynamic-LDS limits of the kernels the plan may use.  A refused request only removes
  // that variant; its error is consumed here so that it does not surface at a later HIP call.
  if (p->variant == VAR_TILE && ckpt_stride > 0 && !p->can_generic) {
    // a checkpointed tile plan solves with its own kernel: the generic solve kernels, whose LDS
    // would hold the generic factor scratch beside the stage (beyond the limit here), are not used
  } else if (lq::prepare_generic(false, p->lds_solve) != hipSuccess) {
    (void)hipGetLastError();
    const size_t need_solve = p->lds_solve;
    (void)hipFree(p->desc_d);  // cleanup of a failed creation
    delete p;
    return fail(LQ_EUNSUPPORTED, "lq_plan_create: cannot reserve %zu bytes of LDS for the solve kernels", need_solve);
  }
  if (p->can_generic && lq::prepare_generic(true, ldsf) != hipSuccess) {
    (void)hipGetLastError();
    p->can_generic = false;
  }
  if (p->can_tile && lq::prepare_tile(p->tile_waves, mode, p->lds_tile) != hipSuccess) {
    (void)hipGetLastError();
    p->can_tile = false;
  }
  if (p->can_tile && ckpt_stride == 0 && lq::tsolve_sizes(p->maxnx, p->maxnu, &p->ts_nxp, &p->ts_nup) &&
      lq::prepare_tsolve(p->ts_nxp, p->ts_nup, mode) != hipSuccess) {
    (void)hipGetLastError();
    p->ts_nxp = p->ts_nup = 0;
  }
  if (p->can_tile && ckpt_stride > 0 && lq::prepare_tckpt(p->ts_nxp, p->ts_nup, mode, p->lds_tckpt) != hipSuccess) {
    (void)hipGetLastError();
    p->can_tile = false;
  }
  // ragged tile plans: one launch per kernel shape (an instance runs with the kernels sized for it,
  // not for the largest instance of the batch)
  if (p->can_tile && ckpt_stride == 0 && p->ts_nxp > 0 && !p->uniform) {
    typedef std::tuple<int, int, int> Key;
    std::map<Key, std::vector<int32_t>> groups;
    std::map<Key, double> gcost;
    for (int32_t i : order) {
      int nxp = 0, nup = 0;
      lq::tsolve_sizes(nx[i], nu[i], &nxp, &nup);
      const Key key(lq::tile_waves((nx[i] + 15) / 16 + (nu[i] + 15) / 16), nxp, nup);
      groups[key].push_back(i);
      gcost[key] += cost[i];
    }
    if (groups.size() > 1) {
      std::vector<Key> keys;
      for (auto& kv : groups) keys.push_back(kv.first);
      std::stable_sort(keys.begin(), keys.end(), [&](const Key& x_, const Key& y_) { return gcost[x_] > gcost[y_]; });
      std::vector<int32_t> border;
      bool ok = true;
      for (const Key& key : keys) {
        lq_plan::Bucket b;
        std::tie(b.waves, b.nxp, b.nup) = key;
        b.off = (int32_t)border.size();
        b.cnt = (int32_t)groups[key].size();
        b.lds_tile = 0;
        for (int32_t i : groups[key]) {
          b.lds_tile = std::max(b.lds_tile, lq::tile_lds_bytes(nx[i], nu[i], mode));
          border.push_back(i);
        }
        b.grid_factor = b.grid_solve = b.cnt;
        if (lq::prepare_tile(b.waves, mode, b.lds_tile) != hipSuccess ||
            lq::prepare_tsolve(b.nxp, b.nup, mode) != hipSuccess) {
          (void)hipGetLastError();
          ok = false;
        }
        p->buckets.push_back(b);
      }
      if (!ok || hipMemcpy(p->border_d, border.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        p->buckets.clear();
      }
      // each group's persistent kernels take their own pair of work counters (2 + 2 i, 3 + 2 i)
      if (2 * p->buckets.size() + 2 > 64) p->buckets.clear();
      if (p->buckets.size() > 1) {
        bool made = true;
        for (size_t i = 0; i < p->buckets.size() && made; ++i) {
          hipEvent_t e = nullptr;
          made = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
          if (made) p->ev.push_back(e);
          if (made && i > 0) {
            hipStream_t st2 = nullptr;
            made = hipStreamCreateWithFlags(&st2, hipStreamNonBlocking) == hipSuccess;
            if (made) p->side.push_back(st2);
          }
        }
        if (!made) {
          (void)hipGetLastError();
          for (hipStream_t x : p->side) (void)hipStreamDestroy(x);
          for (hipEvent_t x : p->ev) (void)hipEventDestroy(x);
          p->side.clear();
          p->ev.clear();
        }
      }
    }
  }
  if ((p->variant == VAR_GENERIC && !p->can_generic) || (p->variant == VAR_TILE && !p->can_tile)) {
    (void)hipFree(p->desc_d);  // cleanup of a failed creation
    delete p;
    return fail(LQ_EUNSUPPORTED, "lq_plan_create: cannot reserve the LDS of the selected kernel");
  }
  p->launch.persistent = p->uniform ? 0 : 1;
  p->launch.threads = p->maxnx + p->maxnu > 48 ? 256 : 128;
  update_grids(p);
  *out = p;
  return LQ_OK;
}

extern "C" int lq_plan_create_subset(const lq_plan* parent, int32_t n, const int32_t* idx, lq_mode mode,
                                     int32_t ckpt_stride, lq_plan** out) {
  g_err.clear();
  const char* fn = "lq_plan_create_subset";
  if (!out) return fail(LQ_EINVAL, "%s: out is NULL", fn);
  *out = nullptr;
  if (!parent || !idx) return fail(LQ_EINVAL, "%s: parent and idx are required", fn);
  if (n <= 0 || n > parent->batch) return fail(LQ_EINVAL, "%s: n = %d outside 1..%d", fn, n, parent->batch);
  std::vector<char> seen(parent->batch, 0);
  std::vector<int32_t> N(n), nx(n), nu(n);
  for (int i = 0; i < n; ++i) {
    const int j = idx[i];
    if (j < 0 || j >= parent->batch) return fail(LQ_EINVAL, "%s: idx[%d] = %d outside the parent's batch", fn, i, j);
    if (seen[j]) return fail(LQ_EINVAL, "%s: instance %d listed twice", fn, j);
    seen[j] = 1;
    N[i] = parent->N[j];
    nx[i] = parent->nx[j];
    nu[i] = parent->nu[j];
  }
  lq_plan* p = nullptr;
  int rc = lq_plan_create(n, N.data(), nx.data(), nu.data(), mode, ckpt_stride, &p);
  if (rc) return rc;
  // the instances live in the parent's arrays: take over its data and output offsets
  for (int i = 0; i < n; ++i) {
    Desc& D = p->desc_h[i];
    const Desc& P = parent->desc_h[idx[i]];
    D.oA = P.oA; D.oB = P.oB; D.oQ = P.oQ; D.oR = P.oR; D.oS = P.oS; D.oq = P.oq; D.or_ = P.or_; D.of = P.of;
    D.ox0 = P.ox0; D.ox = P.ox; D.ou = P.ou; D.olam = P.olam; D.oK = P.oK;
    for (int a = 0; a < LQ_ARR_COUNT; ++a) p->off[a][i] = parent->off[a][idx[i]];
  }
  for (int a = 0; a < LQ_ARR_COUNT; ++a) p->total[a] = parent->total[a];
  p->can_small = p->can_small_pad = false;
  if (p->inner) {  // the padded copies would address the parent's arrays as a dense batch
    lq_plan_destroy(p->inner);
    p->inner = nullptr;
    p->ws_bytes = p->offPad;
  }
  if (p->variant == VAR_SMALL || p->variant == VAR_SMALL_PAD) p->variant = p->can_tile ? VAR_TILE : VAR_GENERIC;
  if (p->variant == VAR_GENERIC && !p->can_generic) {
    lq_plan_destroy(p);
    return fail(LQ_EUNSUPPORTED, "%s: no descriptor-addressed kernel takes these sizes", fn);
  }
  update_grids(p);
  if (hipMemcpy(p->desc_d, p->desc_h.data(), sizeof(Desc) * n, hipMemcpyHostToDevice) != hipSuccess) {
    lq_plan_destroy(p);
    return fail(LQ_EHIP, "%s: descriptor upload failed", fn);
  }
  *out = p;
  return LQ_OK;
}

extern "C" int lq_plan_set_launch(lq_plan* p, const lq_launch* c) {
  g_err.clear();
  if (!p || !c) return fail(LQ_EINVAL, "lq_plan_set_launch: plan and cfg are required");
  if (c->threads != 64 && c->threads != 128 && c->threads != 256 && c->threads != 512)
    return fail(LQ_EINVAL, "lq_plan_set_launch: threads must be 64, 128, 256 or 512");
  if (c->persistent != 0 && c->persistent != 1) return fail(LQ_EINVAL, "lq_plan_set_launch: persistent is 0 or 1");
  if (c->blocks_per_cu < 0 || c->blocks_per_cu > 64)
    return fail(LQ_EINVAL, "lq_plan_set_launch: blocks_per_cu must be in [0, 64]");
  p->launch = *c;
  update_grids(p);
  return LQ_OK;
}

extern "C" int lq_plan_get_launch(const lq_plan* p, lq_launch* c) {
  if (!p || !c) return fail(LQ_EINVAL, "lq_plan_get_launch: plan and cfg are required");
  *c = p->launch;
  return LQ_OK;
}

static lq::GenericLaunch generic_launch(const lq_plan* p, void* ws, bool factor) {
  lq::GenericLaunch c;
  c.threads = p->launch.threads;
  c.order = p->order_d;
  c.counter = nullptr;
  c.grid = p->batch;
  c.ckpt = p->ckpt;
  if (p->launch.persistent) {
    c.grid = factor ? p->grid_factor : p->grid_solve;
    c.counter = (int32_t*)((char*)ws + p->offCtr) + (factor ? 0 : 1);
  }
  return c;
}

// Launch shape of group i's kernels: its slice of the grouped order, its persistent grid, its own
// work counters (the groups may run at the same time).
static lq::GenericLaunch bucket_launch(const lq_plan* p, void* ws, bool factor, size_t i) {
  const lq_plan::Bucket& b = p->buckets[i];
  lq::GenericLaunch c = generic_launch(p, ws, factor);
  c.order = p->border_d + b.off;
  c.grid = p->launch.persistent ? (factor ? b.grid_factor : b.grid_solve) : b.cnt;
  if (c.counter) c.counter = (int32_t*)((char*)ws + p->offCtr) + 2 + 2 * (int)i + (factor ? 0 : 1);
  return c;
}

// Runs launch(i, stream) for every group: the first on the caller's stream, the others on the
// plan's side streams after the fork point, all joined back before the caller's stream goes on.
template <typename F>
static hipError_t run_groups(const lq_plan* p, hipStream_t st, F&& launch) {
  const size_t n = p->buckets.size();
  hipError_t e = hipSuccess;
  if (p->side.empty()) {
    for (size_t i = 0; i < n && e == hipSuccess; ++i) e = launch(i, st);
    return e;
  }
  if ((e = hipEventRecord(p->ev[0], st)) != hipSuccess) return e;
  if ((e = launch((size_t)0, st)) != hipSuccess) return e;
  for (size_t i = 1; i < n; ++i) {
    hipStream_t s2 = p->side[i - 1];
    if ((e = hipStreamWaitEvent(s2, p->ev[0], 0)) != hipSuccess) return e;
    if ((e = launch(i, s2)) != hipSuccess) return e;
    if ((e = hipEventRecord(p->ev[i], s2)) != hipSuccess) return e;
  }
  for (size_t i = 1; i < n; ++i)
    if ((e = hipStreamWaitEvent(st, p->ev[i], 0)) != hipSuccess) return e;
  return hipSuccess;
}

extern "C" int lq_plan_launch_groups(const lq_plan* p) {
  if (!p) return fail(LQ_EINVAL, "lq_plan_launch_groups: plan is NULL");
  return p->variant == VAR_TILE && !p->ckpt && !p->buckets.empty() ? (int)p->buckets.size() : 1;
}

extern "C" void lq_plan_destroy(lq_plan* p) {
  if (!p) return;
  // work of the plan's groups may still run on its streams: let it finish before they go
  for (hipStream_t x : p->side) {
    (void)hipStreamSynchronize(x);
    (void)hipStreamDestroy(x);
  }
  for (hipEvent_t x : p->ev) (void)hipEventDestroy(x);
  if (p->desc_d) (void)hipFree(p->desc_d);
  delete p;
}

extern "C" size_t lq_plan_workspace_bytes(const lq_plan* p) { return p ? p->ws_bytes : 0; }

extern "C" int64_t lq_plan_offsets(const lq_plan* p, lq_array which, int64_t* offs) {
  if (!p || which < 0 || which >= LQ_ARR_COUNT) {
    fail(LQ_EINVAL, "lq_plan_offsets: invalid plan or array");
    return -1;
  }
  if (offs) memcpy(offs, p->off[which].data(), sizeof(int64_t) * p->batch);
  return p->total[which];
}

extern "C" const char* lq_plan_variant(const lq_plan* p) {
  if (!p) return "";
  return p->variant == VAR_SMALL       ? "small"
         : p->variant == VAR_SMALL_PAD ? "small_padded"
         : p->variant == VAR_TILE      ? "tile"
                                       : "generic";
}

extern "C" int lq_plan_set_variant(lq_plan* p, const char* name) {
  g_err.clear();
  if (!p || !name) return fail(LQ_EINVAL, "lq_plan_set_variant: plan and name are required");
  Variant v;
  bool ok;
  if (!strcmp(name, "small")) { v = VAR_SMALL; ok = p->can_small; }
  else if (!strcmp(name, "small_padded")) { v = VAR_SMALL_PAD; ok = p->can_small_pad; }
  else if (!strcmp(name, "tile")) { v = VAR_TILE; ok = p->can_tile; }
  else if (!strcmp(name, "generic")) { v = VAR_GENERIC; ok = p->can_generic; }
  else return fail(LQ_EINVAL, "lq_plan_set_variant: unknown variant '%s'", name);
  if (!ok) return fail(LQ_EUNSUPPORTED, "lq_plan_set_variant: variant '%s' cannot take this plan", name);
  p->variant = v;
  update_grids(p);
  return LQ_OK;
}

static int check_common(const lq_plan* p, const lq_data* d, void* ws, const char* fn) {
  if (!p) return fail(LQ_EINVAL, "%s: plan is NULL", fn);
  if (!d) return fail(LQ_EINVAL, "%s: data is NULL", fn);
  if (!d->A || !d->B || !d->Q || !d->R || !d->q || !d->r || !d->x0)
    return fail(LQ_EINVAL, "%s: A, B, Q, R, q, r, x0 are required", fn);
  if (!ws) return fail(LQ_EINVAL, "%s: workspace is NULL", fn);
  if (((uintptr_t)ws) & 255) return fail(LQ_EINVAL, "%s: workspace must be 256-byte aligned", fn);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(LQ_EINVAL, "%s: current device %d differs from the plan's device %d", fn, dev, p->device);
  return LQ_OK;
}

static int launch_status(hipError_t e, const char* fn) {
  if (e != hipSuccess) return fail(LQ_EHIP, "%s: launch failed: %s", fn, hipGetErrorString(e));
  return LQ_OK;
}

// Padded copies of a VAR_SMALL_PAD plan's data in its workspace (S and f as given: present or NULL).
static lq_data padded_data(const lq_plan* p, const lq_data* d, char* w) {
  lq_data pd;
  pd.A = (const double*)(w + p->offPadArr[0]);
  pd.B = (const double*)(w + p->offPadArr[1]);
  pd.Q = (const double*)(w + p->offPadArr[2]);
  pd.R = (const double*)(w + p->offPadArr[3]);
  pd.S = d->S ? (const double*)(w + p->offPadArr[4]) : nullptr;
  pd.q = (const double*)(w + p->offPadArr[5]);
  pd.r = (const double*)(w + p->offPadArr[6]);
  pd.f = d->f ? (const double*)(w + p->offPadArr[7]) : nullptr;
  pd.x0 = (const double*)(w + p->offPadArr[8]);
  return pd;
}

// lq_factor of a VAR_SMALL_PAD plan: the data padded to the compiled shape, the inner plan's factor
// (its factors, sweep vectors and the padded data stay in this plan's workspace for lq_solve), and
// the factor blocks copied out into this plan's own layout, the one every variant writes (the
// adjoint then runs on the descriptor-addressed kernels, as for size-specialised plans).
static int factor_padded(const lq_plan* p, const lq_data* d, char* w, int32_t* info, hipStream_t st) {
  const int64_t b = p->batch, n = p->N[0];
  const int x = p->nx[0], u = p->nu[0], X = p->pad_nx, U = p->pad_nu;
  lq::PadOp ops[9];
  int k = 0;
  auto add = [&](const double* src, int arr, int64_t blocks, int r, int c, int R, int C, double diag) {
    ops[k++] = lq::PadOp{src, (double*)(w + p->offPadArr[arr]), blocks, r, c, R, C, diag, 0};
  };
  add(d->A, 0, b * n, x, x, X, X, 0.0);
  add(d->B, 1, b * n, x, u, X, U, 0.0);
  add(d->Q, 2, b * (n + 1), x, x, X, X, 1.0);
  add(d->R, 3, b * n, u, u, U, U, 1.0);
  if (d->S) add(d->S, 4, b * n, u, x, U, X, 0.0);
  add(d->q, 5, b * (n + 1), 1, x, 1, X, 0.0);
  add(d->r, 6, b * n, 1, u, 1, U, 0.0);
  if (d->f) add(d->f, 7, b * n, 1, x, 1, X, 0.0);
  add(d->x0, 8, b, 1, x, 1, X, 0.0);
  int rc = launch_status(lq::launch_pad(ops, k, st), "lq_factor");
  if (rc) return rc;
  const lq_data pd = padded_data(p, d, w);
  if ((rc = lq_factor(p->inner, &pd, w + p->offPad, info, st))) return rc;
  return launch_status(lq::launch_extract_small_factors(p->mode == LQ_F64, w + p->offPad + p->inner->offF,
                                                        w + p->offF, b * (n + 1), x, u, X, U, st),
                       "lq_factor");
}

extern "C" int lq_factor(const lq_plan* p, const lq_data* d, void* ws, int32_t* info, hipStream_t st) {
  g_err.clear();
  int rc = check_common(p, d, ws, "lq_factor");
  if (rc) return rc;
  if (!info) return fail(LQ_EINVAL, "lq_factor: info is NULL");
  char* w = (char*)ws;
  if (p->variant == VAR_SMALL_PAD) return factor_padded(p, d, w, info, st);
  void* F = w + p->offF;
  double* V = (double*)(w + p->offV);
  hipError_t e;
  if (p->variant == VAR_SMALL && lq::small_aligned(*d, ws))
    e = lq::launch_factor_small(p->mode, p->batch, p->N[0], p->nx[0], p->nu[0], *d, F, V, info, st);
  else if (p->variant == VAR_TILE && !p->buckets.empty()) {
    e = run_groups(p, st, [&](size_t i, hipStream_t s2) {
      const lq_plan::Bucket& b = p->buckets[i];
      return lq::launch_factor_tile(p->mode, b.waves, p->desc_d, b.cnt, *d, F, V, info, b.lds_tile,
                                    bucket_launch(p, ws, true, i), s2);
    });
  } else if (p->variant == VAR_TILE)
    e = lq::launch_factor_tile(p->mode, p->tile_waves, p->desc_d, p->batch, *d, F, V, info, p->lds_tile,
                               generic_launch(p, ws, true), st);
  else
    e = lq::launch_factor_generic(p->mode, p->desc_d, p->batch, *d, F, V, info, p->lds_factor,
                                  generic_launch(p, ws, true), st);
  return launch_status(e, "lq_factor");
}

static lq::SolveArgs base_args(const lq_plan* p, const lq_data* d, void* ws, const lq_solve_opts* o) {
  char* w = (char*)ws;
  lq::SolveArgs a;
  memset(&a, 0, sizeof a);
  a.desc = p->desc_d;
  a.batch = p->batch;
  a.d = *d;
  a.F = w + p->offF;
  a.V = (const double*)(w + p->offV);
  a.V2 = (double*)(w + p->offV2);
  a.tol = o->tol;
  a.max_it = o->max_it;
  a.check = o->check;
  a.ckpt = p->ckpt;
  a.lds_factor_doubles = (int32_t)(p->lds_factor / sizeof(double));
  a.stage_doubles = (int32_t)p->stage_doubles;
  return a;
}

// Solve kernel of the plan's variant (the size-specialised one is dispatched by the caller).
static hipError_t launch_solve_plan(const lq_plan* p, const lq::SolveArgs& a, void* ws, hipStream_t st) {
  const lq::GenericLaunch c = generic_launch(p, ws, false);
  if (p->variant == VAR_TILE && p->ckpt)
    return lq::launch_solve_tckpt(p->ts_nxp, p->ts_nup, p->mode, a, p->lds_tckpt, c, st);
  if (p->variant == VAR_TILE && !p->buckets.empty()) {
    return run_groups(p, st, [&](size_t i, hipStream_t s2) {
      const lq_plan::Bucket& b = p->buckets[i];
      lq::SolveArgs ab = a;
      ab.batch = b.cnt;
      return lq::launch_solve_tsolve(b.nxp, b.nup, p->mode, ab, bucket_launch(p, ws, false, i), s2);
    });
  }
  if (p->variant == VAR_TILE && p->ts_nxp) return lq::launch_solve_tsolve(p->ts_nxp, p->ts_nup, p->mode, a, c, st);
  return lq::launch_solve_generic(p->mode, a, p->lds_solve, c, st);
}

static int check_opts(const lq_solve_opts* o, const char* fn) {
  if (!o) return fail(LQ_EINVAL, "%s: opts is NULL", fn);
  if (!(o->tol >= 0.0)) return fail(LQ_EINVAL, "%s: tol must be >= 0", fn);
  if (o->max_it < 0 || o->max_it > 1000) return fail(LQ_EINVAL, "%s: max_it must be in [0, 1000]", fn);
  return LQ_OK;
}

extern "C" int lq_solve(const lq_plan* p, const lq_data* d, void* ws, const lq_solve_opts* o, double* x,
                        double* u, double* lam, double* rel_res, int32_t* iters, int32_t* info,
                        hipStream_t st) {
  g_err.clear();
  int rc = check_common(p, d, ws, "lq_solve");
  if (rc) return rc;
  if ((rc = check_opts(o, "lq_solve"))) return rc;
  if (!x || !u || !lam) return fail(LQ_EINVAL, "lq_solve: x, u, lam are required");
  if (!info) return fail(LQ_EINVAL, "lq_solve: info is NULL");
  if (p->variant == VAR_SMALL_PAD) {
    // the inner plan's solve on the padded data lq_factor left in the workspace, then the real
    // rows of x, u, lam (rel_res, iters and info are those of the padded problem, the same values)
    char* w = (char*)ws;
    const lq_data pd = padded_data(p, d, w);
    double* xp = (double*)(w + p->offPadArr[9]);
    double* up = (double*)(w + p->offPadArr[10]);
    double* lp = (double*)(w + p->offPadArr[11]);
    if ((rc = lq_solve(p->inner, &pd, w + p->offPad, o, xp, up, lp, rel_res, iters, info, st))) return rc;
    const int64_t bn = (int64_t)p->batch * p->N[0];
    const int x_ = p->nx[0], u_ = p->nu[0], X = p->pad_nx, U = p->pad_nu;
    const lq::PadOp ops[3] = {{xp, x, bn, 1, x_, 1, X, 0.0, 1}, {up, u, bn, 1, u_, 1, U, 0.0, 1},
                              {lp, lam, bn, 1, x_, 1, X, 0.0, 1}};
    return launch_status(lq::launch_pad(ops, 3, st), "lq_solve");
  }
  lq::SolveArgs a = base_args(p, d, ws, o);
  a.x = x; a.u = u; a.lam = lam;
  a.rhs = lq::RHS_PRIMAL;
  a.rel_res = rel_res; a.iters = iters; a.info = info;
  hipError_t e;
  if (p->variant == VAR_SMALL && lq::small_aligned(*d, ws))
    e = lq::launch_solve_small(p->mode, p->N[0], p->nx[0], p->nu[0], a, st);
  else
    e = launch_solve_plan(p, a, ws, st);
  return launch_status(e, "lq_solve");
}

extern "C" int lq_solve_backward(const lq_plan* p, const lq_data* d, void* ws, const lq_solve_opts* o,
                                 const double* x, const double* u, const double* lam, const double* gx,
                                 const double* gu, double* gA, double* gB, double* gQ, double* gR,
                                 double* gS, double* gq, double* gr, double* gf, double* gx0,
                                 double* rel_res, int32_t* iters, int32_t* info, hipStream_t st) {
  g_err.clear();
  int rc = check_common(p, d, ws, "lq_solve_backward");
  if (rc) return rc;
  if ((rc = check_opts(o, "lq_solve_backward"))) return rc;
  if (!x || !u || !lam || !gx || !gu) return fail(LQ_EINVAL, "lq_solve_backward: x, u, lam, gx, gu are required");
  if (!gA || !gB || !gQ || !gR || !gq || !gr || !gx0)
    return fail(LQ_EINVAL, "lq_solve_backward: gA, gB, gQ, gR, gq, gr, gx0 are required");
  if (!info) return fail(LQ_EINVAL, "lq_solve_backward: info is NULL");
  char* w = (char*)ws;
  double* ZB = (double*)(w + p->offZB);
  lq::SolveArgs a = base_args(p, d, ws, o);
  a.x = ZB;
  a.out_is_zb = 1;
  a.gx = gx; a.gu = gu;
  a.rhs = lq::RHS_ADJOINT;
  a.rel_res = rel_res; a.iters = iters; a.info = info;
  hipError_t e = launch_solve_plan(p, a, ws, st);
  if ((rc = launch_status(e, "lq_solve_backward"))) return rc;
  lq::GradArgs g;
  g.desc = p->desc_d; g.batch = p->batch; g.d = *d;
  g.x = x; g.u = u; g.lam = lam; g.ZB = ZB;
  g.gA = gA; g.gB = gB; g.gQ = gQ; g.gR = gR; g.gS = gS; g.gq = gq; g.gr = gr; g.gf = gf; g.gx0 = gx0;
  e = lq::launch_grad_generic(g, st);
  return launch_status(e, "lq_solve_backward");
}

// ---------------------------------------------------------------------------------------------
// Factorisation updates (lqupdate.h).
static int check_update_rows(const lq_plan* p, const lq_update* u, const char* fn) {
  if (!u || u->m == 0) return LQ_OK;
  if (u->m < 0 || u->m > LQ_UPDATE_MAX_ROWS)
    return fail(LQ_EINVAL, "%s: m = %d outside 0..%d", fn, u->m, LQ_UPDATE_MAX_ROWS);
  if (!u->C || !u->D || !u->dsig) return fail(LQ_EINVAL, "%s: C, D and dsig are required when m > 0", fn);
  return LQ_OK;
}

// Largest stage pieces of a plan for the update kernels: L^R + 1/diag + L^S, L^Q + 1/diag, the
// whole block; and the sums of N nx and N + 1 over the instances.
struct UpdSizes {
  int lrs = 0, lq = 0, fs = 0;
  int64_t sum_Nnx = 0, sum_K = 0;
  int wmax = 0;
};
static UpdSizes update_sizes(const lq_plan* p) {
  UpdSizes z;
  for (int i = 0; i < p->batch; ++i) {
    const int64_t x = p->nx[i], u = p->nu[i];
    z.lrs = (int)std::max<int64_t>(z.lrs, std::min<int64_t>(u * (u + 1) / 2 + u + x * u, 1 << 30));
    z.lq = (int)std::max<int64_t>(z.lq, std::min<int64_t>(x * (x + 1) / 2 + x, 1 << 30));
    z.fs = (int)std::max<int64_t>(z.fs, std::min<int64_t>(lq::stage_factor_elems(x, u), 1 << 30));
    z.sum_Nnx += (int64_t)p->N[i] * x;
    z.sum_K += (int64_t)p->N[i] + 1;
  }
  z.wmax = lq::update_width(z.lrs, z.lq, p->maxnx + p->maxnu, p->maxnx, nullptr);
  return z;
}

extern "C" int32_t lq_update_max_columns(const lq_plan* p) { return p ? update_sizes(p).wmax : 0; }

extern "C" size_t lq_update_workspace_bytes(const lq_plan* p) {
  if (!p) return 0;
  const UpdSizes z = update_sizes(p);
  if (z.wmax <= 0) return 0;
  size_t oSg, oWk, oSt, tot;
  lq::update_ws_layout(z.wmax, z.sum_Nnx, z.sum_K, p->batch, &oSg, &oWk, &oSt, &tot);
  return tot;
}

extern "C" int lq_update_data(const lq_plan* p, const lq_update* u, double* Q, double* R, double* S,
                              hipStream_t st) {
  g_err.clear();
  const char* fn = "lq_update_data";
  if (!p) return fail(LQ_EINVAL, "%s: plan is NULL", fn);
  int rc = check_update_rows(p, u, fn);
  if (rc) return rc;
  if (!Q || !R || !S) return fail(LQ_EINVAL, "%s: Q, R and S are required", fn);
  if (!u || u->m == 0) return LQ_OK;
  return launch_status(lq::launch_update_data(p->desc_d, p->batch, p->maxN, *u, Q, R, S, st), fn);
}

extern "C" int lq_factor_update(const lq_plan* p, const lq_data* d, const lq_update* u, void* ws, void* uws,
                                int32_t* info, hipStream_t st) {
  g_err.clear();
  const char* fn = "lq_factor_update";
  int rc = check_common(p, d, ws, fn);
  if (rc) return rc;
  if (!info) return fail(LQ_EINVAL, "%s: info is NULL", fn);
  if ((rc = check_update_rows(p, u, fn))) return rc;
  if (p->mode != LQ_F64 || p->ckpt != 0)
    return fail(LQ_EUNSUPPORTED, "%s: updates need a float64 plan without checkpoints", fn);
  if (p->variant == VAR_SMALL_PAD)
    return fail(LQ_EUNSUPPORTED, "%s: the factors of a small_padded plan are kept padded; select another variant", fn);
  const UpdSizes z = update_sizes(p);
  const bool rows = u && u->m > 0;
  if (!lq::update_sweep_fits(z.fs, p->maxnx + p->maxnu, p->maxnx) || (rows && z.wmax <= 0))
    return fail(LQ_EUNSUPPORTED, "%s: a stage of this plan does not fit the update kernels' LDS", fn);
  if (rows && !uws) return fail(LQ_EINVAL, "%s: the update workspace is required with update rows", fn);
  if (rows && p->batch > 65535) return fail(LQ_EUNSUPPORTED, "%s: at most 65535 instances with update rows", fn);
  if (rows && (((uintptr_t)uws) & 255)) return fail(LQ_EINVAL, "%s: update workspace must be 256-byte aligned", fn);
  lq_update none = {0, nullptr, nullptr, nullptr};
  char* w = (char*)ws;
  return launch_status(lq::launch_factor_update(p->desc_d, p->batch, p->maxN, z.lrs, z.lq, z.fs, p->maxnx + p->maxnu,
                                                p->maxnx, z.sum_Nnx, z.sum_K, *d, rows ? *u : none,
                                                (double*)(w + p->offF), (double*)(w + p->offV), uws, info, st),
                       fn);
}

// ---------------------------------------------------------------------------------------------
// Box-constrained QPs (lqqp.h): the outer and inner loops on the host, one synchronisation per
// inner step (the loops end when no instance is still iterating).
static void qp_totals(const lq_plan* p, int64_t* tot, int64_t* sumK) {
  const lq_array arr[10] = {LQ_ARR_Q, LQ_ARR_R, LQ_ARR_S, LQ_ARR_q, LQ_ARR_r, LQ_ARR_f, LQ_ARR_x0,
                            LQ_ARR_x, LQ_ARR_u, LQ_ARR_lam};
  for (int i = 0; i < 10; ++i) tot[i] = p->total[arr[i]];
  int64_t k = 0;
  for (int i = 0; i < p->batch; ++i) k += (int64_t)p->N[i] + 1;
  *sumK = k;
}

// The parallel-in-time factors follow the QP workspace's own regions.
static size_t qp_pit_bytes(const lq_plan* p, int32_t P) {
  if (P <= 1) return 0;
  if (!p->uniform) return (size_t)-1;
  return lq_pit_workspace_bytes(p->batch, p->N[0], p->nx[0], p->nu[0], P);
}

extern "C" size_t lq_qp_workspace_bytes(const lq_plan* p, int32_t m, int32_t intervals) {
  if (!p || m <= 0) return 0;
  int64_t tot[10], sumK;
  qp_totals(p, tot, &sumK);
  const size_t pit = qp_pit_bytes(p, intervals);
  if (pit == (size_t)-1 || (intervals > 1 && pit == 0)) return 0;
  return lq::qp_layout(tot, sumK, p->batch, m).total + pit;
}

extern "C" int lq_qp_solve(const lq_plan* p, const lq_data* d, const lq_qp_constraints* c, const lq_qp_opts* o,
                           void* pws, void* qws, double* x, double* u, double* lam, double* y, int32_t* status,
                           int32_t* iters, hipStream_t st) {
  g_err.clear();
  const char* fn = "lq_qp_solve";
  int rc = check_common(p, d, pws, fn);
  if (rc) return rc;
  if (!c || !o) return fail(LQ_EINVAL, "%s: constraints and options are required", fn);
  if (c->m <= 0 || c->m > 256 || !c->C || !c->D || !c->bl || !c->bu)
    return fail(LQ_EINVAL, "%s: m in 1..256 and C, D, bl, bu are required", fn);
  if (!qws || (((uintptr_t)qws) & 255)) return fail(LQ_EINVAL, "%s: a 256-byte aligned QP workspace is required", fn);
  if (!x || !u || !lam || !y || !status || !iters) return fail(LQ_EINVAL, "%s: x, u, lam, y, status, iters are required", fn);
  if (p->mode != LQ_F64 || p->ckpt != 0) return fail(LQ_EUNSUPPORTED, "%s: a float64 plan without checkpoints is required", fn);
  if (p->maxnx > 256) return fail(LQ_EUNSUPPORTED, "%s: nx <= 256", fn);
  if (!(o->sigma0 > 0) || !(o->gamma > 0) || !(o->eps > 0) || o->max_outer <= 0 || o->max_inner <= 0)
    return fail(LQ_EINVAL, "%s: sigma0, gamma, eps, max_outer, max_inner must be positive", fn);
  const int P = o->intervals;
  if (P > 1 && (!p->uniform || P > p->N[0]))
    return fail(LQ_EUNSUPPORTED, "%s: intervals > 1 needs a uniform plan and intervals <= N", fn);
  int64_t tot[10], sumK;
  qp_totals(p, tot, &sumK);
  const lq::QPLayout L = lq::qp_layout(tot, sumK, p->batch, c->m);
  lq::QPArgs a = lq::qp_args(p->desc_d, p->batch, c->m, *d, *c, *o, qws, L, x, u, y);
  char* w = (char*)qws;
  int32_t* finfo = (int32_t*)(w + L.oinfo);
  double* rel = (double*)(w + L.orel);
  int32_t* cnt = (int32_t*)(w + L.ocnt);
  lq_data nd = *d;
  // the iterate is a rollout of the dynamics, so the Newton systems' dynamics right-hand side is
  // zero (f absent)
  nd.Q = a.Qn; nd.R = a.Rn; nd.S = a.Sn; nd.q = a.qn; nd.r = a.rn; nd.f = nullptr; nd.x0 = a.x0n;
  const lq_solve_opts so = {1e-10, 0, 0};
  const int maxN = p->maxN, nxm = p->maxnx, num = p->maxnu;
  hipError_t e = lq::qp_launch(0, a, maxN, nxm, num, st, nullptr, nullptr);
  if (e != hipSuccess) return launch_status(e, fn);
  for (int outer = 0; outer < o->max_outer; ++outer) {
    for (int inner = 0; inner < o->max_inner; ++inner) {
      if ((e = lq::qp_launch(1, a, maxN, nxm, num, st, nullptr, nullptr)) != hipSuccess) return launch_status(e, fn);
      if (P > 1) {
        const int n0 = p->N[0], x0 = p->nx[0], u0 = p->nu[0];
        void* pitws = w + L.total;
        if ((rc = lq_pit_factor(p->batch, n0, x0, u0, P, &nd, pitws, finfo, st))) return rc;
        if ((rc = lq_pit_solve(p->batch, n0, x0, u0, P, &nd, pitws, a.dx, a.du, a.dlam, rel, finfo, st))) return rc;
        // one refinement step with the same factors: the Schur-complement solves lose accuracy at
        // large penalties, which would leave the inner loops with inexact directions
        if ((e = lq::qp_refine(0, a, maxN, nxm, num, tot, st)) != hipSuccess) return launch_status(e, fn);
        lq_data cd = nd;
        cd.q = a.qc; cd.r = a.rc; cd.f = a.fc;
        if ((rc = lq_pit_solve(p->batch, n0, x0, u0, P, &cd, pitws, a.cdx, a.cdu, a.cdlam, rel, finfo, st))) return rc;
        if ((e = lq::qp_refine(1, a, maxN, nxm, num, tot, st)) != hipSuccess) return launch_status(e, fn);
      } else {
        if ((rc = lq_factor(p, &nd, pws, finfo, st))) return rc;
        if ((rc = lq_solve(p, &nd, pws, &so, a.dx, a.du, a.dlam, rel, nullptr, finfo, st))) return rc;
      }
      if ((e = lq::qp_launch(2, a, maxN, nxm, num, st, finfo, cnt)) != hipSuccess) return launch_status(e, fn);
      int32_t running = 0;
      if (hipMemcpyAsync(&running, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(LQ_EHIP, "%s: reading the loop count failed", fn);
      if (running == 0) break;
    }
    if ((e = lq::qp_launch(3, a, maxN, nxm, num, st, nullptr, cnt)) != hipSuccess) return launch_status(e, fn);
    int32_t running = 0;
    if (hipMemcpyAsync(&running, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(LQ_EHIP, "%s: reading the loop count failed", fn);
    if (running == 0) break;
  }
  return launch_status(lq::qp_finish(a, lam, status, iters, st), fn);
}

// ---------------------------------------------------------------------------------------------
// Factor + solve without any allocation, for callers that cannot allocate device memory.  The
// workspace lives in a file-scope device array (one copy per GPU, held until the process ends);
// host code reaches it only through the address hipGetSymbolAddress returns for the current
// device, never through the array's name.

namespace {
constexpr size_t kNoAllocScratchBytes = LQ_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> device address of `scratch`

// Address of this device's copy of `scratch` (looked up once per device, with it current).
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return LQ_OK;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return fail(LQ_EHIP, "lq_factor_solve_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return LQ_OK;
}
}  // namespace

// Scratch bytes a uniform batch needs: factors, sweep vectors, refinement state, each 256-byte aligned.
static size_t noalloc_required_bytes(int32_t batch, int32_t N, int32_t nx, int32_t nu, lq_mode mode) {
  const size_t fb = mode == LQ_F64 ? sizeof(double) : sizeof(float);
  const size_t b = (size_t)batch, n = (size_t)N, x = (size_t)nx, u = (size_t)nu;
  size_t o = align256(b * (n + 1) * (size_t)lq::stage_factor_elems(nx, nu) * fb);  // factors
  o = align256(o + b * (n * u + (n + 1) * x) * sizeof(double));                  // sweep vectors
  o = align256(o + b * (size_t)lq::v2_elems(N, nx, nu) * sizeof(double));        // refinement state
  return o;
}

extern "C" int lq_factor_solve_noalloc(int32_t batch, int32_t N, int32_t nx, int32_t nu, lq_mode mode,
                                       const lq_data* d, const lq_solve_opts* o, double* x, double* u,
                                       double* lam, double* rel_res, int32_t* iters, int32_t* info,
                                       hipStream_t st) {
  g_err.clear();
  const char* fn = "lq_factor_solve_noalloc";
  if (batch <= 0 || N <= 0 || nx <= 0 || nu <= 0)
    return fail(LQ_EINVAL, "%s: batch, N, nx, nu must be positive", fn);
  if (mode != LQ_F64 && mode != LQ_MIXED_F32) return fail(LQ_EUNSUPPORTED, "%s: mode must be LQ_F64 or LQ_MIXED_F32", fn);
  if (!lq::small_variant_available(mode, nx, nu))
    return fail(LQ_EUNSUPPORTED, "%s: no size-specialised kernel for nx=%d nu=%d", fn, nx, nu);
  if (!d || !d->A || !d->B || !d->Q || !d->R || !d->q || !d->r || !d->x0)
    return fail(LQ_EINVAL, "%s: A, B, Q, R, q, r, x0 are required", fn);
  int rc = check_opts(o, fn);
  if (rc) return rc;
  if (!x || !u || !lam || !info) return fail(LQ_EINVAL, "%s: x, u, lam, info are required", fn);
  const size_t need = noalloc_required_bytes(batch, N, nx, nu, mode);
  if (need > kNoAllocScratchBytes)
    return fail(LQ_EUNSUPPORTED, "%s: batch %d x N %d (nx %d, nu %d) needs %zu bytes of scratch, above the %zu available",
                fn, batch, N, nx, nu, need, kNoAllocScratchBytes);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LQ_EHIP, "%s: hipGetDevice failed", fn);
  void* ws = nullptr;
  if ((rc = scratch_address(dev, &ws))) return rc;
  if (!lq::small_aligned(*d, ws)) return fail(LQ_EINVAL, "%s: every data array must be 16-byte aligned", fn);
  const size_t fb = mode == LQ_F64 ? sizeof(double) : sizeof(float);
  char* w = (char*)ws;
  void* F = w;
  double* V = (double*)(w + align256((size_t)batch * (N + 1) * (size_t)lq::stage_factor_elems(nx, nu) * fb));
  double* V2 = (double*)((char*)V + align256((size_t)batch * ((size_t)N * nu + (size_t)(N + 1) * nx) * sizeof(double)));
  hipError_t e = lq::launch_factor_small(mode, batch, N, nx, nu, *d, F, V, info, st);
  if ((rc = launch_status(e, fn))) return rc;
  lq::SolveArgs a;
  memset(&a, 0, sizeof a);
  a.batch = batch;
  a.d = *d;
  a.F = F;
  a.V = V;
  a.V2 = V2;
  a.tol = o->tol;
  a.max_it = o->max_it;
  a.check = o->check;
  a.x = x; a.u = u; a.lam = lam;
  a.rhs = lq::RHS_PRIMAL;
  a.rel_res = rel_res; a.iters = iters; a.info = info;
  e = lq::launch_solve_small(mode, N, nx, nu, a, st);
  return launch_status(e, fn);
}
