// Host runtime behind the C ABI in include/vgicp.h: argument validation,
// contexts, voxel-map and factor-set handles, schedules and HIP graphs.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "vgicp_internal.hpp"

namespace vgicp {
int voxelize_impl(vgicp_ctx ctx, const vgicp_cloud *cloud, double resolution, vgicp_map *out,
                  std::string &msg);
int map_export_impl(vgicp_ctx ctx, vgicp_map m, int32_t *keys, float *mean, float *cov,
                    int32_t *count, std::string &msg);
hipError_t launch_linearize(const vgicp_factorset_s *fs, int accum, int resid, int fused,
                            float kappa, bool lin, int64_t tb, int64_t te, const double *poses, int32_t *corr,
                            hipStream_t st, int32_t stride = 1, const void *consts = nullptr);
hipError_t launch_factor_consts(const vgicp_factorset_s *fs, const double *poses, hipStream_t st);
hipError_t launch_overlap(const vgicp_factorset_s *fs, int64_t tb, int64_t te,
                          const double *poses, hipStream_t st, int32_t stride = 1);
hipError_t launch_reduce(const vgicp_factorset_s *fs, int64_t f0, int64_t nf, const double *poses,
                         int mode, double *H, double *b, double *e, int64_t *inl,
                         double *overlap, hipStream_t st);
hipError_t launch_assemble(const vgicp_factorset_s *fs, const double *H, const double *b,
                           double *Hdiag, double *bvec, double *Hoff, hipStream_t st);
hipError_t linearize_blocks_per_cu(int accum, int fused, int form, int *blocks);
hipError_t launch_linearize_pair(const vgicp_factorset_s *fs, int accum, int resid, int fused,
                                 float kappa, int64_t tb, int64_t te, const double *poses,
                                 hipStream_t st, int32_t stride = 1,
                                 const void *consts = nullptr);
hipError_t launch_reduce_pair(const vgicp_factorset_s *fs, int64_t f0, int64_t nf, double *H,
                              double *b, double *e, int64_t *inl, hipStream_t st);
}  // namespace vgicp

using namespace vgicp;

namespace {

thread_local std::string g_thread_error;

int fail(vgicp_ctx ctx, int code, const std::string &msg) {
  if (ctx)
    ctx->last_error = msg;
  else
    g_thread_error = msg;
  return code;
}

int hip_fail(vgicp_ctx ctx, const char *what, hipError_t e) {
  return fail(ctx, e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

// Make ctx's device current for the calling thread.
int use_device(vgicp_ctx ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, "hipSetDevice", e);
  return VGICP_OK;
}

constexpr int64_t kMinAutoTiles = 3072;  // several tiles per resident block slot

// Tile length of the factors cut into short tiles at the end of an XCD's run
// in the balanced layout: a quarter of tp in whole lookup phases.
int32_t short_tile(int32_t tp) {
  const int32_t q = (tp / 4) / kTileQuantum * kTileQuantum;
  return std::min(tp, std::max(q, int32_t(kTileQuantum)));
}

// Balanced layout: the grouped order cut into 8 runs of about equal points,
// one per XCD (the kernels deal the table to the XCDs in eighths); in each
// run the factors that end in its last tenth of points get short tiles, so
// that the blocks an XCD starts last are short and its CUs finish together;
// the runs are padded to one length with padding tiles.
void build_balanced(vgicp_factorset fs, int32_t tp, std::vector<Tile> &tiles) {
  const std::vector<int64_t> &order = fs->tile_order;
  int64_t total = 0;
  for (int64_t f : order) total += fs->h_factors[size_t(f)].n;
  std::vector<int> run_of(order.size(), 0);
  int64_t run_points[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t before = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    const int64_t n = fs->h_factors[size_t(order[k])].n;
    run_of[k] = total > 0 ? int(std::min<int64_t>(7, before * 8 / total)) : 0;
    run_points[run_of[k]] += n;
    before += n;
  }
  const int32_t tq = short_tile(tp);
  std::vector<Tile> runs[8];
  int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (size_t k = 0; k < order.size(); ++k) {
    const int r = run_of[k];
    FactorDesc &d = fs->h_factors[size_t(order[k])];
    acc[r] += d.n;
    d.tile_points = 10 * acc[r] > 9 * run_points[r] ? tq : tp;
    d.tile_stride = 1;
    d.tile_begin = int32_t(runs[r].size());  // within the run for now
    for (int64_t s = 0; s < d.n; s += d.tile_points)
      runs[r].push_back(Tile{int32_t(order[k]), int32_t(s)});
    d.n_tiles = int32_t(int64_t(runs[r].size()) - d.tile_begin);
  }
  size_t len = 0;
  for (const auto &run : runs) len = std::max(len, run.size());
  tiles.reserve(8 * len);
  for (int r = 0; r < 8; ++r) {
    tiles.insert(tiles.end(), runs[r].begin(), runs[r].end());
    tiles.resize(size_t(r + 1) * len, Tile{kPaddingTile, 0});
  }
  for (size_t k = 0; k < order.size(); ++k)
    fs->h_factors[size_t(order[k])].tile_begin += int32_t(size_t(run_of[k]) * len);
}

// The tile table at `tp` points per tile in the factor set's layout, setting
// every factor's tile_begin, n_tiles, tile_stride and tile_points:
//   VGICP_LAYOUT_GROUPED: factors in tile order (grouped by target map), each
//     factor's tiles consecutive;
//   VGICP_LAYOUT_INTERLEAVED: the factors that read one source copy (the same
//     cloud, unless vgicp_factorset_reorder gave each factor its own copy) side
//     by side, tile by tile (tile p of each such factor, then p + 1, ...), so
//     that tiles streaming the same source points run at the same time on one
//     XCD and share its L2; copies in order of their source cloud;
//   VGICP_LAYOUT_BALANCED: see build_balanced.
void build_tiles(vgicp_factorset fs, int32_t tp, std::vector<Tile> &tiles) {
  tiles.clear();
  if (fs->layout == VGICP_LAYOUT_BALANCED) {
    build_balanced(fs, tp, tiles);
    return;
  }
  if (fs->layout != VGICP_LAYOUT_INTERLEAVED) {
    for (int64_t f : fs->tile_order) {
      FactorDesc &d = fs->h_factors[size_t(f)];
      d.tile_begin = int32_t(tiles.size());
      d.tile_stride = 1;
      d.tile_points = tp;
      for (int64_t s = 0; s < d.n; s += tp) tiles.push_back(Tile{int32_t(f), int32_t(s)});
      d.n_tiles = int32_t(int64_t(tiles.size()) - d.tile_begin);
    }
    return;
  }
  std::vector<int64_t> order = fs->tile_order;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return fs->h_src[size_t(a)] < fs->h_src[size_t(b)]; });
  // group: consecutive factors of one source reading the same copy
  size_t g0 = 0;
  while (g0 < order.size()) {
    const FactorDesc &first = fs->h_factors[size_t(order[g0])];
    size_t g1 = g0 + 1;
    while (g1 < order.size() && fs->h_src[size_t(order[g1])] == fs->h_src[size_t(order[g0])] &&
           fs->h_factors[size_t(order[g1])].xyz == first.xyz)
      ++g1;
    const int32_t K = int32_t(g1 - g0);
    const int64_t T = (first.n + tp - 1) / tp;
    const int32_t base = int32_t(tiles.size());
    for (size_t k = g0; k < g1; ++k) {
      FactorDesc &d = fs->h_factors[size_t(order[k])];
      d.tile_begin = base + int32_t(k - g0);
      d.tile_stride = K;
      d.tile_points = tp;
      d.n_tiles = int32_t(T);
    }
    for (int64_t p = 0; p < T; ++p)
      for (size_t k = g0; k < g1; ++k)
        tiles.push_back(Tile{int32_t(order[k]), int32_t(p * tp)});
    g0 = g1;
  }
}

// Brackets one kernel launch with events when timing is on.
struct TimedLaunch {
  vgicp_ctx ctx;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(vgicp_ctx c, int k) : ctx(c), kind(k) {
    if (!ctx->timing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
        hipEventRecord(a, ctx->stream) != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      a = b = nullptr;
    }
  }
  void done() {
    if (!a) return;
    if (hipEventRecord(b, ctx->stream) == hipSuccess) {
      ctx->pending[kind].emplace_back(a, b);
    } else {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
    a = b = nullptr;
  }
};

hipError_t fold_timing(vgicp_ctx ctx) {
  hipError_t err = hipStreamSynchronize(ctx->stream);
  for (int k = 0; k < VGICP_KERNEL_KINDS; ++k) {
    for (auto &p : ctx->pending[k]) {
      float ms = 0.f;
      if (err == hipSuccess) {
        err = hipEventElapsedTime(&ms, p.first, p.second);
        if (err == hipSuccess) {
          ctx->total_ms[k] += double(ms);
          ctx->launches[k] += 1;
        }
      }
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    ctx->pending[k].clear();
  }
  return err;
}

}  // namespace

int vgicp::set_error(vgicp_ctx ctx, int code, const std::string &msg) {
  return fail(ctx, code, msg);
}

extern "C" {

int vgicp_version(void) { return 200; }

const char *vgicp_last_error(vgicp_ctx ctx) {
  return ctx ? ctx->last_error.c_str() : g_thread_error.c_str();
}

int vgicp_ctx_create(int device, void *hip_stream, vgicp_ctx *out) {
  if (!out) return fail(nullptr, VGICP_EINVAL, "vgicp_ctx_create: out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(nullptr, "vgicp_ctx_create: hipGetDeviceCount", e);
  if (device < 0 || device >= n)
    return fail(nullptr, VGICP_EINVAL, "vgicp_ctx_create: device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, "vgicp_ctx_create: hipSetDevice", e);
  vgicp_ctx ctx = new (std::nothrow) vgicp_context_s();
  if (!ctx) return fail(nullptr, VGICP_ENOMEM, "vgicp_ctx_create: out of host memory");
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  e = hipMalloc(&ctx->err_word, 256);
  if (e == hipSuccess) e = hipHostMalloc(&ctx->host_pinned, 64, hipHostMallocDefault);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, device);
  // the device address of the allocation-free entry point's scratch array
  if (e == hipSuccess) e = noalloc_setup(device);
  if (e != hipSuccess) {
    if (ctx->err_word) (void)hipFree(ctx->err_word);
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    delete ctx;
    return hip_fail(nullptr, "vgicp_ctx_create", e);
  }
  *out = ctx;
  return VGICP_OK;
}

int vgicp_ctx_set_stream(vgicp_ctx ctx, void *hip_stream) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_ctx_set_stream: ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return VGICP_OK;
}

int vgicp_ctx_synchronize(vgicp_ctx ctx) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_ctx_synchronize: ctx is NULL");
  int rc = use_device(ctx);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, "hipStreamSynchronize", e);
  return VGICP_OK;
}

int vgicp_ctx_set_timing(vgicp_ctx ctx, int enable) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_ctx_set_timing: ctx is NULL");
  ctx->timing = enable != 0;
  return VGICP_OK;
}

int vgicp_ctx_read_timing(vgicp_ctx ctx, int kernel, double *total_ms, int64_t *launches) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_ctx_read_timing: ctx is NULL");
  if (kernel < 0 || kernel >= VGICP_KERNEL_KINDS)
    return fail(ctx, VGICP_EINVAL, "vgicp_ctx_read_timing: unknown kernel kind");
  int rc = use_device(ctx);
  if (rc) return rc;
  hipError_t e = fold_timing(ctx);
  if (e != hipSuccess) return hip_fail(ctx, "vgicp_ctx_read_timing", e);
  if (total_ms) *total_ms = ctx->total_ms[kernel];
  if (launches) *launches = ctx->launches[kernel];
  return VGICP_OK;
}

int vgicp_ctx_reset_timing(vgicp_ctx ctx) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_ctx_reset_timing: ctx is NULL");
  int rc = use_device(ctx);
  if (rc) return rc;
  hipError_t e = fold_timing(ctx);
  for (int k = 0; k < VGICP_KERNEL_KINDS; ++k) {
    ctx->total_ms[k] = 0.0;
    ctx->launches[k] = 0;
  }
  if (e != hipSuccess) return hip_fail(ctx, "vgicp_ctx_reset_timing", e);
  return VGICP_OK;
}

int vgicp_ctx_destroy(vgicp_ctx ctx) {
  if (!ctx) return VGICP_OK;
  (void)hipSetDevice(ctx->device);
  (void)fold_timing(ctx);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->map_ws) (void)hipFree(ctx->map_ws);
  if (ctx->map_host) (void)hipHostFree(ctx->map_host);
  if (ctx->err_word) (void)hipFree(ctx->err_word);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  delete ctx;
  return VGICP_OK;
}

// ------------------------------------------------------------------ maps

int vgicp_voxelize(vgicp_ctx ctx, const vgicp_cloud *cloud, double resolution, vgicp_map *out) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_voxelize: ctx is NULL");
  if (!out) return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: out is NULL");
  *out = nullptr;
  if (!cloud) return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: cloud is NULL");
  if (cloud->n < 0) return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: n < 0");
  if (cloud->n > kMaxCloudPoints)
    return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: more than 2^26 points");
  if (cloud->n > 0 && (!cloud->xyz || !cloud->cov))
    return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: NULL point arrays with n > 0");
  if (cloud->n > 0 && (reinterpret_cast<uintptr_t>(cloud->cov) & 7u))
    return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: cov is not 8-byte aligned");
  if (!std::isfinite(resolution) || !(resolution > 0.0))
    return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: resolution must be finite and > 0");
  const float s = float(1.0 / resolution);
  if (!std::isfinite(s) || !(s > 0.0f))
    return fail(ctx, VGICP_EINVAL, "vgicp_voxelize: 1/resolution is not a positive FP32 value");
  int rc = use_device(ctx);
  if (rc) return rc;
  std::string msg;
  rc = voxelize_impl(ctx, cloud, resolution, out, msg);
  if (rc != VGICP_OK) return fail(ctx, rc, msg);
  return VGICP_OK;
}

int vgicp_map_info(vgicp_map map, int64_t *n_voxels, int64_t *capacity, int64_t *device_bytes,
                   double *resolution) {
  if (!map) return fail(nullptr, VGICP_EINVAL, "vgicp_map_info: map is NULL");
  if (n_voxels) *n_voxels = map->n_voxels;
  if (capacity) *capacity = map->capacity;
  if (device_bytes)
    *device_bytes = map->device_bytes();
  if (resolution) *resolution = map->resolution;
  return VGICP_OK;
}

int vgicp_map_export(vgicp_ctx ctx, vgicp_map map, int32_t *keys, float *mean, float *cov,
                     int32_t *count) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_map_export: ctx is NULL");
  if (!map) return fail(ctx, VGICP_EINVAL, "vgicp_map_export: map is NULL");
  if (map->device != ctx->device)
    return fail(ctx, VGICP_EINVAL, "vgicp_map_export: map lives on another device");
  int rc = use_device(ctx);
  if (rc) return rc;
  std::string msg;
  rc = map_export_impl(ctx, map, keys, mean, cov, count, msg);
  if (rc != VGICP_OK) return fail(ctx, rc, msg);
  return VGICP_OK;
}

int vgicp_map_free(vgicp_map map) {
  if (!map) return VGICP_OK;
  (void)hipSetDevice(map->device);
  if (map->buffer) (void)hipFree(map->buffer);
  delete map;
  return VGICP_OK;
}

// ------------------------------------------------------------ factor sets

int vgicp_validate_factors(int32_t n_sources, int32_t n_maps, int32_t n_poses,
                           const vgicp_factor *factors, int64_t n_factors) {
  if (n_sources < 0 || n_maps < 0 || n_poses < 0 || n_factors < 0)
    return fail(nullptr, VGICP_EINVAL, "vgicp_validate_factors: negative count");
  if (n_factors > 0 && !factors)
    return fail(nullptr, VGICP_EINVAL, "vgicp_validate_factors: factors is NULL");
  if (n_factors > INT32_MAX)
    return fail(nullptr, VGICP_EINVAL, "vgicp_validate_factors: more than 2^31-1 factors");
  for (int64_t f = 0; f < n_factors; ++f) {
    const vgicp_factor &x = factors[f];
    const char *bad = nullptr;
    if (x.src < 0 || x.src >= n_sources) bad = "src";
    else if (x.tgt < 0 || x.tgt >= n_maps) bad = "tgt";
    else if (x.pose_i < 0 || x.pose_i >= n_poses) bad = "pose_i";
    else if (x.pose_j < 0 || x.pose_j >= n_poses) bad = "pose_j";
    if (bad)
      return fail(nullptr, VGICP_EINVAL,
                  "vgicp_validate_factors: factor " + std::to_string(f) + " has " + bad +
                      " out of range");
  }
  return VGICP_OK;
}

int vgicp_factorset_create(vgicp_ctx ctx, const vgicp_cloud *sources, int32_t n_sources,
                           const vgicp_map *maps, int32_t n_maps, const vgicp_factor *factors,
                           int64_t n_factors, int32_t n_poses, int32_t tile_points,
                           vgicp_factorset *out) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_create: ctx is NULL");
  if (!out) return fail(ctx, VGICP_EINVAL, "vgicp_factorset_create: out is NULL");
  *out = nullptr;
  if (n_sources > 0 && !sources)
    return fail(ctx, VGICP_EINVAL, "vgicp_factorset_create: sources is NULL");
  if (n_maps > 0 && !maps) return fail(ctx, VGICP_EINVAL, "vgicp_factorset_create: maps is NULL");
  if (vgicp_validate_factors(n_sources, n_maps, n_poses, factors, n_factors) != VGICP_OK)
    return fail(ctx, VGICP_EINVAL, g_thread_error);
  if (tile_points != 0 && (tile_points < 256 || tile_points > (1 << 20) || tile_points % 256 != 0))
    return fail(ctx, VGICP_EINVAL,
                "vgicp_factorset_create: tile_points must be a multiple of 256 in [256, 2^20]");
  for (int32_t s = 0; s < n_sources; ++s) {
    const vgicp_cloud &c = sources[s];
    if (c.n < 0 || c.n > kMaxCloudPoints || (c.n > 0 && (!c.xyz || !c.cov)) ||
        (c.n > 0 && (reinterpret_cast<uintptr_t>(c.cov) & 7u)))
      return fail(ctx, VGICP_EINVAL,
                  "vgicp_factorset_create: source " + std::to_string(s) + " is invalid");
  }
  for (int32_t m = 0; m < n_maps; ++m)
    if (!maps[m] || maps[m]->device != ctx->device)
      return fail(ctx, VGICP_EINVAL,
                  "vgicp_factorset_create: map " + std::to_string(m) + " is NULL or foreign");
  if (tile_points == 0) {
    // Automatic: the default tile, made smaller (in steps of whole lookup
    // phases) while the grid would not give every resident block slot several
    // tiles (small factor sets such as a local submap).
    auto count_tiles = [&](int64_t tp) {
      int64_t t = 0;
      for (int64_t f = 0; f < n_factors; ++f) t += (sources[factors[f].src].n + tp - 1) / tp;
      return t;
    };
    tile_points = kDefaultTile;
    for (int q : {6, 4, 3, 2, 1}) {
      tile_points = q * kTileQuantum;
      if (count_tiles(tile_points) >= kMinAutoTiles) break;
    }
  }
  int rc = use_device(ctx);
  if (rc) return rc;

  auto *fs = new (std::nothrow) vgicp_factorset_s();
  if (!fs) return fail(ctx, VGICP_ENOMEM, "vgicp_factorset_create: out of host memory");
  fs->device = ctx->device;
  fs->n_factors = n_factors;
  fs->n_poses = n_poses;
  fs->tile_points = tile_points;
  fs->h_factors.resize(size_t(n_factors));

  // Ordered copies of the source clouds that factors use, in cells of the
  // finest resolution among the maps each cloud is matched against.
  std::vector<SortedSource> sorted;
  {
    std::vector<double> cell(size_t(n_sources), 0.0);
    for (int64_t f = 0; f < n_factors; ++f) {
      double &c = cell[size_t(factors[f].src)];
      const double r = maps[factors[f].tgt]->resolution;
      c = (c == 0.0) ? r : std::min(c, r);
    }
    int64_t nonfinite[2] = {0, 0};
    const hipError_t se = make_sorted_sources(sources, n_sources, cell, &fs->d_sorted, sorted,
                                              ctx->stream, nonfinite);
    fs->nonfinite_points = nonfinite[0];
    fs->nonfinite_covs = nonfinite[1];
    if (se != hipSuccess) {
      vgicp_factorset_destroy(fs);
      return hip_fail(ctx, "vgicp_factorset_create", se);
    }
  }

  // Tile order: factors grouped by target map so that consecutive tiles (and
  // therefore one XCD's share of the grid) reuse the same hash table.
  std::vector<int64_t> order(static_cast<size_t>(n_factors));
  std::iota(order.begin(), order.end(), int64_t(0));
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return factors[a].tgt < factors[b].tgt;
  });
  int64_t corr_off = 0;
  for (int64_t f = 0; f < n_factors; ++f) {
    const vgicp_factor &x = factors[f];
    FactorDesc &d = fs->h_factors[size_t(f)];
    std::memset(&d, 0, sizeof(d));
    const vgicp_cloud &c = sources[x.src];
    const vgicp_voxelmap_s *m = maps[x.tgt];
    const SortedSource &ss = sorted[size_t(x.src)];
    d.xyz = ss.xyz ? ss.xyz : c.xyz;
    d.cov = ss.xyz ? ss.cov : c.cov;
    d.perm = ss.perm;
    d.bricks = m->bricks;
    d.stats = m->stats;
    d.occ = m->occ;
    d.occ_mask = occ_bits(m->capacity) - 1u;
    d.info = m->info;
    d.n = c.n;
    d.corr_offset = corr_off;
    d.pose_i = x.pose_i;
    d.pose_j = x.pose_j;
    d.log2cap = m->log2cap;
    d.scale = m->scale;
    d.n_voxels = uint32_t(m->n_voxels);
    corr_off += c.n;
  }
  fs->total_points = corr_off;
  fs->tile_order = order;
  fs->h_src.resize(size_t(n_factors));
  for (int64_t f = 0; f < n_factors; ++f) fs->h_src[size_t(f)] = factors[f].src;
  std::vector<Tile> tiles;
  build_tiles(fs, tile_points, tiles);
  fs->n_tiles = int64_t(tiles.size());
  fs->tiles_capacity = std::max<int64_t>(1, fs->n_tiles);

  // CSR of system-assembly contributions (factor order within each pose/pair)
  std::vector<int64_t> pose_off(size_t(n_poses) + 1, 0), pose_ent;
  {
    std::vector<std::vector<int64_t>> per(static_cast<size_t>(n_poses));
    for (int64_t f = 0; f < n_factors; ++f) {
      const bool self = factors[f].pose_i == factors[f].pose_j;
      per[size_t(factors[f].pose_i)].push_back(4 * f + (self ? 2 : 0));
      per[size_t(factors[f].pose_j)].push_back(4 * f + 1);
    }
    for (int32_t p = 0; p < n_poses; ++p) {
      pose_off[size_t(p) + 1] = pose_off[size_t(p)] + int64_t(per[size_t(p)].size());
      pose_ent.insert(pose_ent.end(), per[size_t(p)].begin(), per[size_t(p)].end());
    }
  }
  std::vector<int64_t> pair_off(1, 0), pair_ent;
  {
    std::vector<std::pair<std::pair<int32_t, int32_t>, int64_t>> keyed;
    for (int64_t f = 0; f < n_factors; ++f) {
      const int32_t i = factors[f].pose_i, j = factors[f].pose_j;
      if (i == j) continue;
      keyed.push_back({{std::min(i, j), std::max(i, j)}, 2 * f + (i > j ? 1 : 0)});
    }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const auto &x, const auto &y) { return x.first < y.first; });
    for (size_t k = 0; k < keyed.size(); ++k) {
      if (k > 0 && keyed[k].first != keyed[k - 1].first) pair_off.push_back(int64_t(k));
      if (k == 0 || keyed[k].first != keyed[k - 1].first) {
        fs->h_pairs.push_back(keyed[k].first.first);
        fs->h_pairs.push_back(keyed[k].first.second);
      }
      pair_ent.push_back(keyed[k].second);
    }
    if (!keyed.empty()) pair_off.push_back(int64_t(keyed.size()));
    fs->n_pairs = int64_t(fs->h_pairs.size() / 2);
  }

  hipError_t e = hipSuccess;
  const size_t fbytes = std::max<size_t>(1, fs->h_factors.size()) * sizeof(FactorDesc);
  const size_t tbytes = std::max<size_t>(1, tiles.size()) * sizeof(Tile);
  const size_t pbytes = std::max<size_t>(1, tiles.size()) * kPartialStride * sizeof(double);
  e = hipMalloc(&fs->d_factors, fbytes);
  if (e == hipSuccess)
    e = hipMalloc(&fs->d_consts, std::max<size_t>(1, fs->h_factors.size()) * kFactorConstsBytes);
  if (e == hipSuccess) e = hipMalloc(&fs->d_tiles, tbytes);
  if (e == hipSuccess) e = hipMalloc(&fs->d_partials, pbytes);
  // zeroed so that the FP64-point count reads 0 before the first call
  if (e == hipSuccess) e = hipMemsetAsync(fs->d_partials, 0, pbytes, ctx->stream);
  if (e == hipSuccess && n_factors > 0)
    e = hipMemcpyAsync(fs->d_factors, fs->h_factors.data(), fs->h_factors.size() * sizeof(FactorDesc),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpyAsync(fs->d_tiles, tiles.data(), tiles.size() * sizeof(Tile),
                       hipMemcpyHostToDevice, ctx->stream);
  auto upload = [&](int64_t **d, const std::vector<int64_t> &h) {
    if (e != hipSuccess) return;
    e = hipMalloc(d, std::max<size_t>(1, h.size()) * sizeof(int64_t));
    if (e == hipSuccess && !h.empty())
      e = hipMemcpyAsync(*d, h.data(), h.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                         ctx->stream);
  };
  upload(&fs->d_pose_off, pose_off);
  upload(&fs->d_pose_ent, pose_ent);
  upload(&fs->d_pair_off, pair_off);
  upload(&fs->d_pair_ent, pair_ent);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    vgicp_factorset_destroy(fs);
    return hip_fail(ctx, "vgicp_factorset_create", e);
  }
  *out = fs;
  return VGICP_OK;
}

}  // extern "C"

namespace {

// Rebuild the tile table for `tp` points per tile in the factor set's layout
// (build_tiles), growing the device tables when needed.  Captured graphs refer to the
// old table and grid, so they are dropped.  Synchronizes ctx's stream.
int set_tiles(vgicp_ctx ctx, vgicp_factorset fs, int32_t tp, const char *who) {
  std::vector<Tile> tiles;
  build_tiles(fs, tp, tiles);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  for (auto &g : fs->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  fs->graphs.clear();
  const int64_t nt = int64_t(tiles.size());
  if (e == hipSuccess && nt > fs->tiles_capacity) {
    (void)hipFree(fs->d_tiles);
    (void)hipFree(fs->d_partials);
    fs->d_tiles = nullptr;
    fs->d_partials = nullptr;
    fs->tiles_capacity = 0;
    e = hipMalloc(&fs->d_tiles, size_t(nt) * sizeof(Tile));
    if (e == hipSuccess)
      e = hipMalloc(&fs->d_partials, size_t(nt) * kPartialStride * sizeof(double));
    if (e == hipSuccess)
      e = hipMemsetAsync(fs->d_partials, 0, size_t(nt) * kPartialStride * sizeof(double),
                         ctx->stream);
    if (e == hipSuccess) fs->tiles_capacity = nt;
  }
  if (e == hipSuccess && fs->n_factors > 0)
    e = hipMemcpyAsync(fs->d_factors, fs->h_factors.data(),
                       fs->h_factors.size() * sizeof(FactorDesc), hipMemcpyHostToDevice,
                       ctx->stream);
  if (e == hipSuccess && nt > 0)
    e = hipMemcpyAsync(fs->d_tiles, tiles.data(), size_t(nt) * sizeof(Tile),
                       hipMemcpyHostToDevice, ctx->stream);
  // padding tiles keep zero partials (no kernel writes them; the counters
  // sum every tile's row)
  if (e == hipSuccess && nt > 0)
    e = hipMemsetAsync(fs->d_partials, 0, size_t(nt) * kPartialStride * sizeof(double),
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, who, e);
  fs->n_tiles = nt;
  fs->tile_points = tp;
  return VGICP_OK;
}

}  // namespace

extern "C" {

int vgicp_factorset_info(vgicp_factorset fs, int64_t *n_factors, int64_t *n_tiles,
                         int64_t *total_points, int32_t *tile_points) {
  if (!fs) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_info: fs is NULL");
  if (tile_points) *tile_points = fs->tile_points;
  if (n_factors) *n_factors = fs->n_factors;
  if (n_tiles) *n_tiles = fs->n_tiles;
  if (total_points) *total_points = fs->total_points;
  return VGICP_OK;
}

int vgicp_factorset_graph_count(vgicp_factorset fs, int64_t *n_graphs) {
  if (!fs) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_graph_count: fs is NULL");
  if (!n_graphs) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_graph_count: n_graphs is NULL");
  *n_graphs = int64_t(fs->graphs.size());
  return VGICP_OK;
}

int vgicp_factorset_destroy(vgicp_factorset fs) {
  if (!fs) return VGICP_OK;
  (void)hipSetDevice(fs->device);
  for (auto &g : fs->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (fs->d_factors) (void)hipFree(fs->d_factors);
  if (fs->d_consts) (void)hipFree(fs->d_consts);
  if (fs->d_tiles) (void)hipFree(fs->d_tiles);
  if (fs->d_partials) (void)hipFree(fs->d_partials);
  if (fs->d_partials_pair) (void)hipFree(fs->d_partials_pair);
  if (fs->d_sorted) (void)hipFree(fs->d_sorted);
  for (int64_t *p : {fs->d_pose_off, fs->d_pose_ent, fs->d_pair_off, fs->d_pair_ent})
    if (p) (void)hipFree(p);
  delete fs;
  return VGICP_OK;
}

}  // extern "C"

// ----------------------------------------------------------- execution

namespace {

constexpr int kKindLinearize = 0;
constexpr int kKindEvaluate = 1;

}  // namespace

int vgicp::check_common(vgicp_ctx ctx, vgicp_factorset fs, const double *poses, const char *who) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, std::string(who) + ": ctx is NULL");
  if (!fs) return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set is NULL");
  if (fs->device != ctx->device)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set lives on another device");
  if (fs->n_factors > 0 && fs->n_poses > 0 && !poses)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": poses is NULL");
  return use_device(ctx);
}

int vgicp::read_opts(vgicp_ctx ctx, const vgicp_opts *opts, vgicp_opts *o, const char *who) {
  *o = vgicp_opts{VGICP_ACC_MIXED, VGICP_SCHED_BATCHED, 0, VGICP_RESID_F64, 0.0f,
                  VGICP_FUSED_F64, VGICP_FORM_AUTO};
  if (opts) *o = *opts;
  if (o->accum != VGICP_ACC_MIXED && o->accum != VGICP_ACC_F32 && o->accum != VGICP_ACC_F64 &&
      o->accum != VGICP_ACC_F32_COMP)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": unknown accumulation");
  if (o->schedule != VGICP_SCHED_BATCHED && o->schedule != VGICP_SCHED_PER_FACTOR)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": unknown schedule");
  if (o->resid != VGICP_RESID_F64 && o->resid != VGICP_RESID_F32)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": unknown residual mode");
  if (!(o->fp64_kappa >= 0.0f) || !std::isfinite(o->fp64_kappa))
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": fp64_kappa must be finite and >= 0");
  if (o->fused != VGICP_FUSED_F64 && o->fused != VGICP_FUSED_F32)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": unknown fused-covariance precision");
  if (o->form != VGICP_FORM_AUTO && o->form != VGICP_FORM_SOURCE && o->form != VGICP_FORM_PAIR)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": unknown form");
  if (o->form == VGICP_FORM_PAIR && o->accum == VGICP_ACC_F64)
    return fail(ctx, VGICP_EINVAL,
                std::string(who) + ": the pair form accumulates in FP32 per lane (mixed, f32 "
                                   "or f32_comp)");
  return VGICP_OK;
}

namespace {

// The form a linearization runs in: opts' form, or under VGICP_FORM_AUTO the
// factor set's where the pair form applies.
int resolve_form(const vgicp_factorset_s *fs, const vgicp_opts &o, const int32_t *corr) {
  if (o.form != VGICP_FORM_AUTO) return o.form;
  if (fs->form == VGICP_FORM_PAIR && !corr && o.accum != VGICP_ACC_F64) return VGICP_FORM_PAIR;
  return VGICP_FORM_SOURCE;
}

void drop_graphs(vgicp_factorset fs) {
  for (auto &g : fs->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  fs->graphs.clear();
}

// The pair form's tile partials, allocated at its first call and again when
// the tiles have outgrown them (captured graphs hold the old buffer and are
// dropped after the stream's pending work).
int ensure_pair_partials(vgicp_ctx ctx, vgicp_factorset fs, const char *who) {
  if (fs->d_partials_pair && fs->pair_capacity >= fs->n_tiles) return VGICP_OK;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, who, e);
  drop_graphs(fs);
  if (fs->d_partials_pair) (void)hipFree(fs->d_partials_pair);
  fs->d_partials_pair = nullptr;
  fs->pair_capacity = 0;
  const int64_t nt = std::max<int64_t>(std::max(fs->tiles_capacity, fs->n_tiles), 1);
  e = hipMalloc(&fs->d_partials_pair, size_t(nt) * kPairStride * sizeof(double));
  if (e != hipSuccess) return hip_fail(ctx, who, e);
  fs->pair_capacity = nt;
  return VGICP_OK;
}

// Enqueue the factors' tiles [tb, te) and the reduce of factors [f0, f0+nf).
// `ctx` is NULL inside graph capture (no timing events there).
hipError_t enqueue_range(vgicp_ctx ctx, vgicp_factorset fs, int kind, int accum, int resid,
                         int fused, float kappa, const double *poses, int64_t tb, int64_t te, int64_t f0, int64_t nf,
                         double *H, double *b, double *e, int64_t *inl, int32_t *corr,
                         hipStream_t st, int form = VGICP_FORM_SOURCE, int32_t stride = 1) {
  const int tk = kind == kKindLinearize ? VGICP_KERNEL_LINEARIZE : VGICP_KERNEL_EVALUATE;
  hipError_t err = hipSuccess;
  // a launch over the whole tile table reads the factors' constants from a
  // table written once for the round; a launch over one factor's tiles
  // computes them in every tile
  const void *consts = nullptr;
  if (tb == 0 && te == fs->n_tiles && f0 == 0 && nf == fs->n_factors && fs->d_consts) {
    err = launch_factor_consts(fs, poses, st);
    if (err != hipSuccess) return err;
    consts = fs->d_consts;
  }
  if (form == VGICP_FORM_PAIR && kind == kKindLinearize) {
    if (ctx) {
      TimedLaunch t(ctx, tk);
      err = launch_linearize_pair(fs, accum, resid, fused, kappa, tb, te, poses, st, stride,
                                  consts);
      t.done();
    } else {
      err = launch_linearize_pair(fs, accum, resid, fused, kappa, tb, te, poses, st, stride,
                                  consts);
    }
    if (err != hipSuccess) return err;
    if (ctx) {
      TimedLaunch t(ctx, VGICP_KERNEL_REDUCE);
      err = launch_reduce_pair(fs, f0, nf, H, b, e, inl, st);
      t.done();
    } else {
      err = launch_reduce_pair(fs, f0, nf, H, b, e, inl, st);
    }
    return err;
  }
  if (ctx) {
    TimedLaunch t(ctx, tk);
    err = launch_linearize(fs, accum, resid, fused, kappa, kind == kKindLinearize, tb, te, poses, corr,
                           st, stride, consts);
    t.done();
  } else {
    err = launch_linearize(fs, accum, resid, fused, kappa, kind == kKindLinearize, tb, te, poses, corr,
                           st, stride, consts);
  }
  if (err != hipSuccess) return err;
  if (ctx) {
    TimedLaunch t(ctx, VGICP_KERNEL_REDUCE);
    err = launch_reduce(fs, f0, nf, poses, kind, H, b, e, inl, nullptr, st);
    t.done();
  } else {
    err = launch_reduce(fs, f0, nf, poses, kind, H, b, e, inl, nullptr, st);
  }
  return err;
}

int run_factors(vgicp_ctx ctx, vgicp_factorset fs, int kind, const double *poses,
                const vgicp_opts &o, double *H, double *b, double *e, int64_t *inl,
                int32_t *corr, const char *who) {
  if (fs->n_factors == 0) return VGICP_OK;
  hipStream_t st = ctx->stream;
  hipError_t err = hipSuccess;
  if (o.form == VGICP_FORM_PAIR && corr && kind == kKindLinearize)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": the pair form writes no correspondences");
  const int form = kind == kKindLinearize ? resolve_form(fs, o, corr) : VGICP_FORM_SOURCE;
  if (form == VGICP_FORM_PAIR) {
    const int rc = ensure_pair_partials(ctx, fs, who);
    if (rc) return rc;
  }
  if (o.schedule == VGICP_SCHED_PER_FACTOR) {
    for (int64_t f = 0; f < fs->n_factors && err == hipSuccess; ++f) {
      const FactorDesc &d = fs->h_factors[size_t(f)];
      err = enqueue_range(ctx, fs, kind, o.accum, o.resid, o.fused, o.fp64_kappa, poses, d.tile_begin,
                          int64_t(d.tile_begin) + d.n_tiles, f, 1, H, b, e, inl, corr, st, form,
                          d.tile_stride);
    }
    if (err != hipSuccess) return hip_fail(ctx, who, err);
    return VGICP_OK;
  }
  if (!o.use_graph) {
    err = enqueue_range(ctx, fs, kind, o.accum, o.resid, o.fused, o.fp64_kappa, poses, 0, fs->n_tiles, 0, fs->n_factors, H, b, e,
                        inl, corr, st, form);
    if (err != hipSuccess) return hip_fail(ctx, who, err);
    return VGICP_OK;
  }
  if (st == nullptr)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": graph replay needs a non-default stream");
  GraphEntry *g = nullptr;
  for (auto &x : fs->graphs)
    if (x.poses == poses && x.H == H && x.b == b && x.e == e && x.inl == inl && x.corr == corr &&
        x.accum == o.accum && x.resid == o.resid && x.fused == o.fused &&
        x.kappa == o.fp64_kappa && x.kind == kind && x.form == form)
      g = &x;
  if (!g && fs->graphs.size() >= kMaxGraphs) {
    // drop the least recently replayed graph (after its last launch is done)
    size_t lru = 0;
    for (size_t k = 1; k < fs->graphs.size(); ++k)
      if (fs->graphs[k].last_use < fs->graphs[lru].last_use) lru = k;
    err = hipStreamSynchronize(st);
    if (err != hipSuccess) return hip_fail(ctx, who, err);
    (void)hipGraphExecDestroy(fs->graphs[lru].exec);
    (void)hipGraphDestroy(fs->graphs[lru].graph);
    fs->graphs.erase(fs->graphs.begin() + std::ptrdiff_t(lru));
  }
  if (!g) {
    GraphEntry ng{poses, H, b, e, inl, corr, o.accum, o.resid, o.fused, o.fp64_kappa, kind, form};
    err = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) return hip_fail(ctx, "hipStreamBeginCapture", err);
    hipError_t lerr = enqueue_range(nullptr, fs, kind, o.accum, o.resid, o.fused, o.fp64_kappa, poses, 0, fs->n_tiles, 0,
                                    fs->n_factors, H, b, e, inl, corr, st, form);
    err = hipStreamEndCapture(st, &ng.graph);
    if (lerr != hipSuccess) {
      if (ng.graph) (void)hipGraphDestroy(ng.graph);
      return hip_fail(ctx, who, lerr);
    }
    if (err != hipSuccess) return hip_fail(ctx, "hipStreamEndCapture", err);
    err = hipGraphInstantiate(&ng.exec, ng.graph, nullptr, nullptr, 0);
    if (err != hipSuccess) {
      (void)hipGraphDestroy(ng.graph);
      return hip_fail(ctx, "hipGraphInstantiate", err);
    }
    fs->graphs.push_back(ng);
    g = &fs->graphs.back();
  }
  g->last_use = ++fs->graph_clock;
  err = hipGraphLaunch(g->exec, st);
  if (err != hipSuccess) return hip_fail(ctx, "hipGraphLaunch", err);
  return VGICP_OK;
}

}  // namespace

extern "C" {

int vgicp_linearize_factors(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                            const vgicp_opts *opts, double *H, double *b, double *e,
                            int64_t *inliers, int32_t *corr) {
  const char *who = "vgicp_linearize_factors";
  int rc = check_common(ctx, fs, poses, who);
  if (rc) return rc;
  vgicp_opts o;
  rc = read_opts(ctx, opts, &o, who);
  if (rc) return rc;
  if (fs->n_factors > 0 && (!H || !b || !e || !inliers))
    return fail(ctx, VGICP_EINVAL, "vgicp_linearize_factors: an output pointer is NULL");
  return run_factors(ctx, fs, kKindLinearize, poses, o, H, b, e, inliers, corr, who);
}

int vgicp_evaluate_errors(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                          const vgicp_opts *opts, double *e, int64_t *inliers) {
  const char *who = "vgicp_evaluate_errors";
  int rc = check_common(ctx, fs, poses, who);
  if (rc) return rc;
  vgicp_opts o;
  rc = read_opts(ctx, opts, &o, who);
  if (rc) return rc;
  if (fs->n_factors > 0 && (!e || !inliers))
    return fail(ctx, VGICP_EINVAL, "vgicp_evaluate_errors: an output pointer is NULL");
  return run_factors(ctx, fs, kKindEvaluate, poses, o, nullptr, nullptr, e, inliers, nullptr, who);
}

int vgicp_overlap(vgicp_ctx ctx, vgicp_factorset fs, const double *poses, int64_t *hits,
                  double *overlap) {
  const char *who = "vgicp_overlap";
  int rc = check_common(ctx, fs, poses, who);
  if (rc) return rc;
  if (fs->n_factors == 0) return VGICP_OK;
  if (!hits) return fail(ctx, VGICP_EINVAL, "vgicp_overlap: hits is NULL");
  hipError_t err;
  {
    TimedLaunch t(ctx, VGICP_KERNEL_OVERLAP);
    err = launch_overlap(fs, 0, fs->n_tiles, poses, ctx->stream);
    t.done();
  }
  if (err == hipSuccess) {
    TimedLaunch t(ctx, VGICP_KERNEL_REDUCE);
    err = launch_reduce(fs, 0, fs->n_factors, poses, 2, nullptr, nullptr, nullptr, hits, overlap,
                        ctx->stream);
    t.done();
  }
  if (err != hipSuccess) return hip_fail(ctx, who, err);
  return VGICP_OK;
}

}  // extern "C"

extern "C" {

int vgicp_factorset_pairs(vgicp_factorset fs, int64_t *n_pairs, int32_t *pairs) {
  if (!fs) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_pairs: fs is NULL");
  if (n_pairs) *n_pairs = fs->n_pairs;
  if (pairs && fs->n_pairs > 0)
    std::memcpy(pairs, fs->h_pairs.data(), fs->h_pairs.size() * sizeof(int32_t));
  return VGICP_OK;
}

int vgicp_assemble_system(vgicp_ctx ctx, vgicp_factorset fs, const double *H, const double *b,
                          double *Hdiag, double *bvec, double *Hoff) {
  const char *who = "vgicp_assemble_system";
  if (!ctx) return fail(nullptr, VGICP_EINVAL, std::string(who) + ": ctx is NULL");
  if (!fs) return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set is NULL");
  if (fs->device != ctx->device)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set lives on another device");
  if (fs->n_factors > 0 && (!H || !b))
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": H or b is NULL");
  if (fs->n_poses > 0 && (!Hdiag || !bvec))
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": Hdiag or bvec is NULL");
  int rc = use_device(ctx);
  if (rc) return rc;
  hipError_t e = launch_assemble(fs, H, b, Hdiag, bvec, Hoff, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, who, e);
  return VGICP_OK;
}

}  // extern "C"

extern "C" {

int vgicp_factorset_tune(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                         const vgicp_opts *opts, double *H, double *b, double *e,
                         int64_t *inliers, const int32_t *candidates, int32_t n_candidates,
                         int32_t *best_tile, double *best_ms) {
  const char *who = "vgicp_factorset_tune";
  int rc = check_common(ctx, fs, poses, who);
  if (rc) return rc;
  vgicp_opts o;
  rc = read_opts(ctx, opts, &o, who);
  if (rc) return rc;
  if (fs->n_factors > 0 && (!H || !b || !e || !inliers))
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": an output pointer is NULL");
  static const int32_t kDefaultCandidates[] = {42 * kTileQuantum, 30 * kTileQuantum,
                                               24 * kTileQuantum, 18 * kTileQuantum,
                                               12 * kTileQuantum, 6 * kTileQuantum,
                                               4 * kTileQuantum,  3 * kTileQuantum,
                                               2 * kTileQuantum,  kTileQuantum};
  if (!candidates) {
    candidates = kDefaultCandidates;
    n_candidates = int32_t(sizeof(kDefaultCandidates) / sizeof(kDefaultCandidates[0]));
  }
  if (n_candidates < 1)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": no candidate tile sizes");
  for (int32_t k = 0; k < n_candidates; ++k)
    if (candidates[k] < 256 || candidates[k] > (1 << 20) || candidates[k] % 256 != 0)
      return fail(ctx, VGICP_EINVAL,
                  std::string(who) + ": tile sizes must be multiples of 256 in [256, 2^20]");
  o.schedule = VGICP_SCHED_BATCHED;
  o.use_graph = 0;
  // The first rounds after idle run at lower clocks: warm up first, then time
  // every candidate twice (forward and reverse order) and keep its best.
  for (int r = 0; r < 10 && rc == VGICP_OK; ++r)
    rc = run_factors(ctx, fs, kKindLinearize, poses, o, H, b, e, inliers, nullptr, who);
  if (rc != VGICP_OK) return rc;
  const int kWarm = 2, kTimed = 5;
  std::vector<double> cand_ms(size_t(n_candidates), 1e300);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t he = hipEventCreate(&t0);
  if (he == hipSuccess) he = hipEventCreate(&t1);
  if (he != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_fail(ctx, who, he);
  }
  // forms to time: both under VGICP_FORM_AUTO where the pair form applies
  int forms[2] = {o.form == VGICP_FORM_AUTO ? VGICP_FORM_SOURCE : o.form, VGICP_FORM_PAIR};
  const int n_forms = (o.form == VGICP_FORM_AUTO && o.accum != VGICP_ACC_F64) ? 2 : 1;
  // the persistent grid of each form: as many blocks as the CUs hold at once
  int32_t persist[2] = {8, 8};
  for (int fi = 0; fi < n_forms; ++fi) {
    int per_cu = 0;
    he = linearize_blocks_per_cu(o.accum, o.fused, forms[fi], &per_cu);
    if (he != hipSuccess) {
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      return hip_fail(ctx, who, he);
    }
    persist[fi] = std::max(8, (ctx->cu_count * std::max(per_cu, 1)) / 8 * 8);
  }
  // layouts to time: grouped and balanced, and interleaved when some source
  // copy is read by several factors
  const int32_t layout0 = fs->layout;
  const int32_t layouts[3] = {VGICP_LAYOUT_GROUPED, VGICP_LAYOUT_BALANCED,
                              VGICP_LAYOUT_INTERLEAVED};
  int n_layouts = 2;
  {
    std::vector<const float *> copies;
    copies.reserve(fs->h_factors.size());
    for (const FactorDesc &d : fs->h_factors) copies.push_back(d.xyz);
    std::sort(copies.begin(), copies.end());
    if (std::adjacent_find(copies.begin(), copies.end()) != copies.end()) n_layouts = 3;
  }
  // slot (layout, form, candidate, grid) -> best mean round time
  const int32_t n_cfg = n_layouts * n_candidates;
  std::vector<double> grid_ms(size_t(2 * n_forms * n_cfg), 1e300);
  auto slot_of = [&](int li, int fi, int32_t k, int g) {
    return size_t(((li * n_forms + fi) * n_candidates + k) * 2 + g);
  };
  for (int32_t step = 0; step < 2 * n_cfg && rc == VGICP_OK; ++step) {
    const bool fwd = step < n_cfg;
    const int32_t c = fwd ? step : 2 * n_cfg - 1 - step;
    const int li = c / n_candidates;
    const int32_t k = c % n_candidates;
    fs->layout = layouts[li];
    rc = set_tiles(ctx, fs, candidates[k], who);
    for (int q = 0; q < 2 * n_forms && rc == VGICP_OK; ++q) {
      const int qq = fwd ? q : 2 * n_forms - 1 - q;
      const int fi = qq / 2, g = qq % 2;
      vgicp_opts of = o;
      of.form = forms[fi];
      fs->persist_blocks = g ? persist[fi] : 0;
      for (int r = 0; r < kWarm + kTimed && rc == VGICP_OK; ++r) {
        if (r == kWarm && (he = hipEventRecord(t0, ctx->stream)) != hipSuccess)
          rc = hip_fail(ctx, who, he);
        if (rc == VGICP_OK)
          rc = run_factors(ctx, fs, kKindLinearize, poses, of, H, b, e, inliers, nullptr, who);
      }
      float ms = 0.f;
      if (rc == VGICP_OK && (he = hipEventRecord(t1, ctx->stream)) != hipSuccess)
        rc = hip_fail(ctx, who, he);
      if (rc == VGICP_OK && (he = hipEventSynchronize(t1)) != hipSuccess)
        rc = hip_fail(ctx, who, he);
      if (rc == VGICP_OK && (he = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess)
        rc = hip_fail(ctx, who, he);
      const size_t slot = slot_of(li, fi, k, g);
      if (rc == VGICP_OK) grid_ms[slot] = std::min(grid_ms[slot], double(ms) / kTimed);
    }
  }
  size_t best_slot = 0;
  for (size_t q = 1; q < grid_ms.size(); ++q)
    if (grid_ms[q] < grid_ms[best_slot]) best_slot = q;
  const int best_g = int(best_slot % 2);
  const int32_t best = candidates[(best_slot / 2) % size_t(n_candidates)];
  const int best_fi = int((best_slot / size_t(2 * n_candidates)) % size_t(n_forms));
  const int best_li = int(best_slot / size_t(2 * n_candidates * n_forms));
  const double best_t = grid_ms[best_slot];
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  fs->persist_blocks = 0;
  if (rc != VGICP_OK) {
    fs->layout = layout0;
    (void)set_tiles(ctx, fs, fs->tile_points, who);
    return rc;
  }
  fs->layout = layouts[best_li];
  rc = set_tiles(ctx, fs, best, who);
  if (rc != VGICP_OK) return rc;
  fs->persist_blocks = best_g ? persist[best_fi] : 0;
  if (o.form == VGICP_FORM_AUTO) fs->form = forms[best_fi];
  if (best_tile) *best_tile = best;
  if (best_ms) *best_ms = best_t;
  return VGICP_OK;
}

int vgicp_factorset_time_kernel(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                                const vgicp_opts *opts, int32_t kernel, int32_t reps,
                                double *avg_ms) {
  const char *who = "vgicp_factorset_time_kernel";
  int rc = check_common(ctx, fs, poses, who);
  if (rc) return rc;
  vgicp_opts o;
  rc = read_opts(ctx, opts, &o, who);
  if (rc) return rc;
  if (kernel != VGICP_KERNEL_LINEARIZE && kernel != VGICP_KERNEL_EVALUATE &&
      kernel != VGICP_KERNEL_OVERLAP)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": kernel must be linearize, evaluate or overlap");
  if (reps < 1 || reps > 10000)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": reps must be in [1, 10000]");
  if (!avg_ms) return fail(ctx, VGICP_EINVAL, std::string(who) + ": avg_ms is NULL");
  *avg_ms = 0.0;
  if (fs->n_tiles == 0) return VGICP_OK;
  const bool pair =
      kernel == VGICP_KERNEL_LINEARIZE && resolve_form(fs, o, nullptr) == VGICP_FORM_PAIR;
  if (pair) {
    rc = ensure_pair_partials(ctx, fs, who);
    if (rc) return rc;
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  // the round's constants table, written before the timed launches (a round
  // writes it once before its linearize launch)
  hipError_t e = kernel == VGICP_KERNEL_OVERLAP ? hipSuccess
                                                : launch_factor_consts(fs, poses, ctx->stream);
  const void *consts = kernel == VGICP_KERNEL_OVERLAP ? nullptr : fs->d_consts;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e == hipSuccess) e = hipEventRecord(t0, ctx->stream);
  for (int32_t r = 0; r < reps && e == hipSuccess; ++r) {
    if (kernel == VGICP_KERNEL_OVERLAP)
      e = launch_overlap(fs, 0, fs->n_tiles, poses, ctx->stream);
    else if (pair)
      e = launch_linearize_pair(fs, o.accum, o.resid, o.fused, o.fp64_kappa, 0, fs->n_tiles, poses,
                                ctx->stream, 1, consts);
    else
      e = launch_linearize(fs, o.accum, o.resid, o.fused, o.fp64_kappa,
                           kernel == VGICP_KERNEL_LINEARIZE, 0, fs->n_tiles, poses, nullptr,
                           ctx->stream, 1, consts);
  }
  if (e == hipSuccess) e = hipEventRecord(t1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) return hip_fail(ctx, who, e);
  *avg_ms = double(ms) / reps;
  return VGICP_OK;
}

int vgicp_factorset_set_grid(vgicp_ctx ctx, vgicp_factorset fs, int32_t persist_blocks) {
  const char *who = "vgicp_factorset_set_grid";
  if (!ctx) return fail(nullptr, VGICP_EINVAL, std::string(who) + ": ctx is NULL");
  if (!fs) return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set is NULL");
  if (fs->device != ctx->device)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set lives on another device");
  if (persist_blocks < 0 || persist_blocks % 8 != 0 || persist_blocks > (1 << 24))
    return fail(ctx, VGICP_EINVAL,
                std::string(who) + ": persist_blocks must be 0 or a multiple of 8 up to 2^24");
  int rc = use_device(ctx);
  if (rc) return rc;
  if (persist_blocks == fs->persist_blocks) return VGICP_OK;
  // captured graphs hold the old grid: drop them after their last replay
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, who, e);
  for (auto &g : fs->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  fs->graphs.clear();
  fs->persist_blocks = persist_blocks;
  return VGICP_OK;
}

int vgicp_factorset_grid(vgicp_factorset fs, int32_t *persist_blocks) {
  if (!fs) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_grid: factor set is NULL");
  if (persist_blocks) *persist_blocks = fs->persist_blocks;
  return VGICP_OK;
}

int vgicp_factorset_form(vgicp_factorset fs, int32_t *form) {
  if (!fs) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_form: factor set is NULL");
  if (form) *form = fs->form;
  return VGICP_OK;
}

int vgicp_factorset_set_layout(vgicp_ctx ctx, vgicp_factorset fs, int32_t layout) {
  const char *who = "vgicp_factorset_set_layout";
  if (!ctx) return fail(nullptr, VGICP_EINVAL, std::string(who) + ": ctx is NULL");
  if (!fs) return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set is NULL");
  if (fs->device != ctx->device)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set lives on another device");
  if (layout != VGICP_LAYOUT_GROUPED && layout != VGICP_LAYOUT_INTERLEAVED &&
      layout != VGICP_LAYOUT_BALANCED)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": unknown layout");
  int rc = use_device(ctx);
  if (rc) return rc;
  if (layout == fs->layout) return VGICP_OK;
  const int32_t old = fs->layout;
  fs->layout = layout;
  rc = set_tiles(ctx, fs, fs->tile_points, who);
  if (rc != VGICP_OK) fs->layout = old;
  return rc;
}

int vgicp_factorset_layout(vgicp_factorset fs, int32_t *layout) {
  if (!fs) return fail(nullptr, VGICP_EINVAL, "vgicp_factorset_layout: factor set is NULL");
  if (layout) *layout = fs->layout;
  return VGICP_OK;
}

int vgicp_factorset_reorder(vgicp_ctx ctx, vgicp_factorset fs, const double *poses) {
  const char *who = "vgicp_factorset_reorder";
  int rc = check_common(ctx, fs, poses, who);
  if (rc) return rc;
  if (fs->total_points > int64_t(INT32_MAX))
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": more than 2^31 - 1 source points");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = reorder_by_target(fs, poses, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, who, e);
  // captured graphs read the descriptors at run time, but drop them anyway so
  // that no graph outlives the copies it was captured with
  for (auto &g : fs->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  fs->graphs.clear();
  return VGICP_OK;
}

namespace {

// Sum over the factor set's tiles of one slot of the tile partials (a count
// written by the last linearize or evaluate call); synchronizes.
int partial_column_sum(vgicp_ctx ctx, vgicp_factorset fs, int slot, int64_t *total,
                       const char *who) {
  *total = 0;
  if (fs->n_tiles == 0) return VGICP_OK;
  std::vector<double> col(size_t(fs->n_tiles));
  hipError_t e = hipMemcpy2DAsync(col.data(), sizeof(double), fs->d_partials + slot,
                                  kPartialStride * sizeof(double), sizeof(double),
                                  size_t(fs->n_tiles), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess)
    return fail(ctx, VGICP_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  int64_t sum = 0;
  for (double v : col) sum += int64_t(v);
  *total = sum;
  return VGICP_OK;
}

int check_fs(vgicp_ctx ctx, vgicp_factorset fs, const char *who) {
  if (!ctx) return fail(nullptr, VGICP_EINVAL, std::string(who) + ": ctx is NULL");
  if (!fs) return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set is NULL");
  if (fs->device != ctx->device)
    return fail(ctx, VGICP_EINVAL, std::string(who) + ": factor set lives on another device");
  return use_device(ctx);
}

}  // namespace

int vgicp_factorset_fp64_points(vgicp_ctx ctx, vgicp_factorset fs, int64_t *n_points) {
  const char *who = "vgicp_factorset_fp64_points";
  int rc = check_fs(ctx, fs, who);
  if (rc) return rc;
  if (!n_points) return fail(ctx, VGICP_EINVAL, std::string(who) + ": n_points is NULL");
  return partial_column_sum(ctx, fs, kWideSlot, n_points, who);
}

int vgicp_factorset_check(vgicp_ctx ctx, vgicp_factorset fs, int64_t *nonfinite_points,
                          int64_t *nonfinite_covs, int64_t *degenerate_hits) {
  const char *who = "vgicp_factorset_check";
  int rc = check_fs(ctx, fs, who);
  if (rc) return rc;
  if (nonfinite_points) *nonfinite_points = fs->nonfinite_points;
  if (nonfinite_covs) *nonfinite_covs = fs->nonfinite_covs;
  if (degenerate_hits) return partial_column_sum(ctx, fs, kDegenerateSlot, degenerate_hits, who);
  return VGICP_OK;
}

}  // extern "C"
