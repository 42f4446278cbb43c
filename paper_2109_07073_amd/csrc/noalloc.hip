// Linearization into caller-owned outputs with no device allocation.
//
// vgicp_linearize_factors keeps the per-tile partial sums of a round in its
// factor set's own buffer.  vgicp_linearize_factors_noalloc runs the same two
// kernels (k_linearize over the tiles, k_reduce over the factors) but keeps
// the partials in `scratch`, a fixed array of this file with room for
// kScratchTiles tiles, so the call itself allocates nothing.  Each device that
// loads the library holds its own copy of the array until the process ends;
// its address on a device is looked up once, when the first context on that
// device is created.

#include <mutex>

#include "vgicp_internal.hpp"

namespace vgicp {
hipError_t launch_linearize_into(const vgicp_factorset_s *fs, int accum, int resid, int fused,
                                 float kappa, bool lin, int64_t tb, int64_t te,
                                 const double *poses, double *partials, int32_t *corr,
                                 hipStream_t st, int32_t stride = 1,
                                 const void *consts = nullptr);
hipError_t launch_reduce_from(const vgicp_factorset_s *fs, int64_t f0, int64_t nf,
                              const double *poses, const double *partials, int mode, double *H,
                              double *b, double *e, int64_t *inl, double *overlap,
                              hipStream_t st);
}  // namespace vgicp

using namespace vgicp;

namespace {

// Tile partials the array holds: 32,768 tiles of kPartialStride doubles (8 MiB).
constexpr int64_t kScratchTiles = VGICP_NOALLOC_MAX_TILES;
static_assert(kScratchTiles * kPartialStride * sizeof(double) == (size_t(8) << 20),
              "scratch size");

// The array's name is a host-side stand-in: kernels get its device address
// (g_scratch below), never the name.
static __device__ __align__(256) double scratch[kScratchTiles * kPartialStride];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

}  // namespace

hipError_t vgicp::noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = p;
  return hipSuccess;
}

extern "C" {

int vgicp_linearize_factors_noalloc(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                                    const vgicp_opts *opts, double *H, double *b, double *e,
                                    int64_t *inliers, int32_t *corr) {
  const char *who = "vgicp_linearize_factors_noalloc";
  int rc = check_common(ctx, fs, poses, who);
  if (rc) return rc;
  vgicp_opts o;
  rc = read_opts(ctx, opts, &o, who);
  if (rc) return rc;
  if (o.use_graph)
    return set_error(ctx, VGICP_EINVAL,
                     std::string(who) + ": use_graph must be 0 (capturing a graph allocates)");
  if (o.form == VGICP_FORM_PAIR)
    return set_error(ctx, VGICP_EINVAL,
                     std::string(who) + ": the scratch array holds source-frame partials only "
                                        "(form must be VGICP_FORM_AUTO or VGICP_FORM_SOURCE)");
  if (fs->n_factors > 0 && (!H || !b || !e || !inliers))
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": an output pointer is NULL");
  if (fs->n_tiles > kScratchTiles)
    return set_error(ctx, VGICP_ERANGE,
                     std::string(who) + ": the factor set has " + std::to_string(fs->n_tiles) +
                         " tiles, more than the " + std::to_string(kScratchTiles) +
                         " the fixed scratch holds (use larger tiles or "
                         "vgicp_linearize_factors)");
  if (fs->n_factors == 0) return VGICP_OK;
  double *partials = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices)
      partials = static_cast<double *>(g_scratch[ctx->device]);
  }
  if (!partials)
    return set_error(ctx, VGICP_EHIP,
                     std::string(who) + ": no scratch address for this device (context setup "
                                        "failed to look it up)");
  // Every slot the reduce reads is written by the linearize launch before it
  // on the same stream, so nothing needs clearing between calls.
  hipStream_t st = ctx->stream;
  hipError_t err = hipSuccess;
  if (o.schedule == VGICP_SCHED_PER_FACTOR) {
    for (int64_t f = 0; f < fs->n_factors && err == hipSuccess; ++f) {
      const FactorDesc &d = fs->h_factors[size_t(f)];
      const int64_t tb = d.tile_begin, te = int64_t(d.tile_begin) + d.n_tiles;
      err = launch_linearize_into(fs, o.accum, o.resid, o.fused, o.fp64_kappa, true, tb, te, poses,
                                  partials, corr, st, d.tile_stride);
      if (err == hipSuccess)
        err = launch_reduce_from(fs, f, 1, poses, partials, 0, H, b, e, inliers, nullptr, st);
    }
  } else {
    err = launch_linearize_into(fs, o.accum, o.resid, o.fused, o.fp64_kappa, true, 0, fs->n_tiles, poses,
                                partials, corr, st);
    if (err == hipSuccess)
      err = launch_reduce_from(fs, 0, fs->n_factors, poses, partials, 0, H, b, e, inliers,
                               nullptr, st);
  }
  if (err != hipSuccess)
    return set_error(ctx, VGICP_EHIP, std::string(who) + ": " + hipGetErrorString(err));
  return VGICP_OK;
}

}  // extern "C"
