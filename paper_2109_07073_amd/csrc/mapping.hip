// Keyframe control by voxel overlap (vgicp_connect, vgicp_submap_step and
// their server forms in include/vgicp.h).
//
// Paper: Sec. III-B (local mapping: a frame whose overlap with the submap's
// last frame exceeds th^L_max is skipped; the submap closes once the overlap
// between its first and newest frames falls below th^L_min or it holds more
// than N^L_max frames) and Sec. III-C (global mapping: a matching-cost factor
// joins the new submap and every earlier one whose overlap exceeds th^G_min).
// The overlap is Eqs. (7)-(8), counted by the same k_overlap kernel as
// vgicp_overlap; only the comparisons with the thresholds run on the host.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "vgicp_internal.hpp"

namespace vgicp {
hipError_t launch_overlap(const vgicp_factorset_s *fs, int64_t tb, int64_t te,
                          const double *poses, hipStream_t st, int32_t stride = 1);
hipError_t launch_reduce(const vgicp_factorset_s *fs, int64_t f0, int64_t nf, const double *poses,
                         int mode, double *H, double *b, double *e, int64_t *inl,
                         double *overlap, hipStream_t st);
}  // namespace vgicp

using namespace vgicp;

namespace {

constexpr int kOverlapTile = kDefaultTile;  // source points per overlap tile
constexpr size_t kAlign = 256;

size_t aligned(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

bool finite_pose(const double *p) {
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(p[k])) return false;
  return true;
}

int grow(vgicp_ctx ctx, size_t dev_bytes, size_t host_bytes, const char *who) {
  if (ctx->map_ws_bytes < dev_bytes) {
    if (ctx->map_ws) (void)hipFree(ctx->map_ws);
    ctx->map_ws = nullptr;
    ctx->map_ws_bytes = 0;
    const size_t want = std::max(dev_bytes, size_t(1) << 20);
    const hipError_t e = hipMalloc(&ctx->map_ws, want);
    if (e != hipSuccess)
      return set_error(ctx, e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP,
                       std::string(who) + ": " + hipGetErrorString(e));
    ctx->map_ws_bytes = want;
  }
  if (ctx->map_host_bytes < host_bytes) {
    if (ctx->map_host) (void)hipHostFree(ctx->map_host);
    ctx->map_host = nullptr;
    ctx->map_host_bytes = 0;
    const size_t want = std::max(host_bytes, size_t(1) << 20);
    const hipError_t e = hipHostMalloc(&ctx->map_host, want, hipHostMallocDefault);
    if (e != hipSuccess)
      return set_error(ctx, e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP,
                       std::string(who) + ": " + hipGetErrorString(e));
    ctx->map_host_bytes = want;
  }
  return VGICP_OK;
}

// Overlap (Eqs. (7)-(8)) of one cloud at `pose` against n maps at their
// poses: hits[k] points of the cloud fall in a voxel of maps[k] under
// T_k^-1 T, overlap[k] = hits[k] / N (0 for an empty cloud).  Synchronous on
// ctx's stream.  Arguments are validated by the caller.
int overlap_of_cloud(vgicp_ctx ctx, const vgicp_cloud &c, const double *pose,
                     const vgicp_map *maps, const double *map_poses, int32_t n, int64_t *hits,
                     double *overlap, const char *who) {
  if (n == 0) return VGICP_OK;
  const int64_t tiles_per = (c.n + kOverlapTile - 1) / kOverlapTile;
  const int64_t nt = tiles_per * n;
  // device: descriptors, tiles, poses, partials, hits, overlap, then the
  // cloud's coordinates point by point (the layout k_overlap reads)
  const size_t b_desc = aligned(sizeof(FactorDesc) * size_t(n));
  const size_t b_tile = aligned(sizeof(Tile) * size_t(std::max<int64_t>(nt, 1)));
  const size_t b_pose = aligned(sizeof(double) * 12 * size_t(n + 1));
  const size_t b_part = aligned(sizeof(double) * kPartialStride * size_t(std::max<int64_t>(nt, 1)));
  const size_t b_hits = aligned(sizeof(int64_t) * size_t(n));
  const size_t b_ov = aligned(sizeof(double) * size_t(n));
  const size_t b_xyz = aligned(sizeof(float) * 3 * size_t(c.n));
  const size_t dev = b_desc + b_tile + b_pose + b_part + b_hits + b_ov + b_xyz;
  const size_t host = b_desc + b_tile + b_pose + b_hits + b_ov;
  int rc = grow(ctx, dev, host, who);
  if (rc) return rc;
  char *d = static_cast<char *>(ctx->map_ws);
  char *h = static_cast<char *>(ctx->map_host);
  auto *h_desc = reinterpret_cast<FactorDesc *>(h);
  auto *h_tile = reinterpret_cast<Tile *>(h + b_desc);
  auto *h_pose = reinterpret_cast<double *>(h + b_desc + b_tile);
  auto *h_hits = reinterpret_cast<int64_t *>(h + b_desc + b_tile + b_pose);
  auto *h_ov = reinterpret_cast<double *>(h + b_desc + b_tile + b_pose + b_hits);
  auto *d_desc = reinterpret_cast<FactorDesc *>(d);
  auto *d_tile = reinterpret_cast<Tile *>(d + b_desc);
  auto *d_pose = reinterpret_cast<double *>(d + b_desc + b_tile);
  auto *d_part = reinterpret_cast<double *>(d + b_desc + b_tile + b_pose);
  auto *d_hits = reinterpret_cast<int64_t *>(d + b_desc + b_tile + b_pose + b_part);
  auto *d_ov = reinterpret_cast<double *>(d + b_desc + b_tile + b_pose + b_part + b_hits);
  auto *d_xyz = reinterpret_cast<float *>(d + b_desc + b_tile + b_pose + b_part + b_hits + b_ov);

  // the pinned staging may still be read by an earlier call's copies
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return set_error(ctx, VGICP_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  std::memcpy(h_pose, pose, 12 * sizeof(double));
  std::memcpy(h_pose + 12, map_poses, size_t(n) * 12 * sizeof(double));
  int64_t t = 0;
  for (int32_t k = 0; k < n; ++k) {
    const vgicp_voxelmap_s *m = maps[k];
    FactorDesc &fd = h_desc[k];
    std::memset(&fd, 0, sizeof(fd));
    fd.xyz = d_xyz;
    fd.cov = c.cov;
    fd.bricks = m->bricks;
    fd.stats = m->stats;
    fd.info = m->info;
    fd.occ = m->occ;
    fd.occ_mask = occ_bits(m->capacity) - 1u;
    fd.n = c.n;
    fd.pose_i = 0;
    fd.pose_j = k + 1;
    fd.log2cap = m->log2cap;
    fd.scale = m->scale;
    fd.n_voxels = uint32_t(m->n_voxels);
    fd.tile_begin = int32_t(t);
    for (int64_t s = 0; s < c.n; s += kOverlapTile) h_tile[t++] = Tile{k, int32_t(s)};
    fd.n_tiles = int32_t(t - fd.tile_begin);
    fd.tile_stride = 1;
    fd.tile_points = kOverlapTile;
  }
  vgicp_factorset_s view;
  view.device = ctx->device;
  view.n_factors = n;
  view.n_tiles = nt;
  view.tile_points = kOverlapTile;
  view.d_factors = d_desc;
  view.d_tiles = d_tile;
  view.d_partials = d_part;
  const hipStream_t st = ctx->stream;
  e = hipMemcpyAsync(d, h, b_desc + b_tile + b_pose, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_interleave_xyz(c.xyz, c.n, d_xyz, st);
  if (e == hipSuccess) e = launch_overlap(&view, 0, nt, d_pose, st);
  if (e == hipSuccess)
    e = launch_reduce(&view, 0, n, d_pose, 2, nullptr, nullptr, nullptr, d_hits, d_ov, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_hits, d_hits, b_hits + b_ov, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  view.d_factors = nullptr;  // the view owns nothing
  view.d_tiles = nullptr;
  view.d_partials = nullptr;
  if (e != hipSuccess) return set_error(ctx, VGICP_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  if (hits) std::memcpy(hits, h_hits, size_t(n) * sizeof(int64_t));
  if (overlap) std::memcpy(overlap, h_ov, size_t(n) * sizeof(double));
  return VGICP_OK;
}

int check_cloud(vgicp_ctx ctx, const vgicp_cloud *c, const char *who) {
  if (!c) return set_error(ctx, VGICP_EINVAL, std::string(who) + ": cloud is NULL");
  if (c->n < 0 || c->n > kMaxCloudPoints)
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": cloud size outside [0, 2^26]");
  if (c->n > 0 && !c->xyz)
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": cloud xyz is NULL");
  return VGICP_OK;
}

int check_map(vgicp_ctx ctx, vgicp_map m, const char *who) {
  if (!m) return set_error(ctx, VGICP_EINVAL, std::string(who) + ": a map is NULL");
  if (m->device != ctx->device)
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": a map lives on another device");
  return VGICP_OK;
}

int check_rules(const vgicp_submap_rules *r, std::string &msg) {
  if (!r) {
    msg = "rules is NULL";
    return VGICP_EINVAL;
  }
  if (!std::isfinite(r->skip_above) || !std::isfinite(r->close_below) || r->max_frames < 1 ||
      r->reserved != 0) {
    msg = "rules need finite thresholds, max_frames >= 1 and reserved = 0";
    return VGICP_EINVAL;
  }
  return VGICP_OK;
}

bool admitted_by(double overlap, double threshold, int32_t rule) {
  return rule == VGICP_GATE_AT_LEAST ? overlap >= threshold : overlap > threshold;
}

// The local-mapping decision for a frame arriving at a submap of n_submap
// frames, from its overlap with the submap's last and first frames.
int32_t submap_decision(const vgicp_submap_rules &r, int32_t n_submap, double ov_last,
                        double ov_first) {
  if (n_submap == 0) return VGICP_SUBMAP_START;
  if (ov_last > r.skip_above) return VGICP_SUBMAP_SKIP;
  if (ov_first < r.close_below || n_submap + 1 > r.max_frames) return VGICP_SUBMAP_CLOSE;
  return VGICP_SUBMAP_INSERT;
}

}  // namespace

extern "C" {

int vgicp_connect(vgicp_ctx ctx, const vgicp_cloud *cloud, const double *h_pose,
                  const vgicp_map *maps, const double *h_map_poses, int32_t n_maps,
                  double threshold, int32_t rule, int64_t *h_hits, double *h_overlap,
                  int32_t *h_admitted, int32_t *n_admitted) {
  const char *who = "vgicp_connect";
  if (!ctx) return set_error(nullptr, VGICP_EINVAL, std::string(who) + ": ctx is NULL");
  int rc = check_cloud(ctx, cloud, who);
  if (rc) return rc;
  if (n_maps < 0 || (n_maps > 0 && (!maps || !h_map_poses)))
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": bad map list");
  if (!h_pose || !finite_pose(h_pose))
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": pose is NULL or not finite");
  if (!std::isfinite(threshold) || (rule != VGICP_GATE_ABOVE && rule != VGICP_GATE_AT_LEAST))
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": bad threshold or rule");
  if (n_maps > 0 && !h_admitted)
    return set_error(ctx, VGICP_EINVAL, std::string(who) + ": admitted is NULL");
  for (int32_t k = 0; k < n_maps; ++k) {
    rc = check_map(ctx, maps[k], who);
    if (rc) return rc;
    if (!finite_pose(h_map_poses + 12 * size_t(k)))
      return set_error(ctx, VGICP_EINVAL, std::string(who) + ": a map pose is not finite");
  }
  if (hipSetDevice(ctx->device) != hipSuccess)
    return set_error(ctx, VGICP_EHIP, std::string(who) + ": hipSetDevice");
  std::vector<int64_t> hits(size_t(std::max(n_maps, 1)));
  std::vector<double> ov(size_t(std::max(n_maps, 1)));
  rc = overlap_of_cloud(ctx, *cloud, h_pose, maps, h_map_poses, n_maps, hits.data(), ov.data(),
                        who);
  if (rc) return rc;
  int32_t count = 0;
  for (int32_t k = 0; k < n_maps; ++k) {
    h_admitted[k] = admitted_by(ov[size_t(k)], threshold, rule) ? 1 : 0;
    count += h_admitted[k];
    if (h_hits) h_hits[k] = hits[size_t(k)];
    if (h_overlap) h_overlap[k] = ov[size_t(k)];
  }
  if (n_admitted) *n_admitted = count;
  return VGICP_OK;
}

int vgicp_submap_step(vgicp_ctx ctx, const vgicp_submap_rules *rules, const vgicp_cloud *frame,
                      const double *h_pose, vgicp_map first, const double *h_first_pose,
                      vgicp_map last, const double *h_last_pose, int32_t n_submap,
                      int32_t *decision, double *overlap_first, double *overlap_last) {
  const char *who = "vgicp_submap_step";
  if (!ctx) return set_error(nullptr, VGICP_EINVAL, std::string(who) + ": ctx is NULL");
  std::string msg;
  if (check_rules(rules, msg)) return set_error(ctx, VGICP_EINVAL, std::string(who) + ": " + msg);
  int rc = check_cloud(ctx, frame, who);
  if (rc) return rc;
  if (!decision) return set_error(ctx, VGICP_EINVAL, std::string(who) + ": decision is NULL");
  if (n_submap < 0) return set_error(ctx, VGICP_EINVAL, std::string(who) + ": n_submap < 0");
  double ov[2] = {0.0, 0.0};  // last, first
  if (n_submap > 0) {
    if (!h_pose || !finite_pose(h_pose) || !h_first_pose || !finite_pose(h_first_pose) ||
        !h_last_pose || !finite_pose(h_last_pose))
      return set_error(ctx, VGICP_EINVAL, std::string(who) + ": a pose is NULL or not finite");
    if ((rc = check_map(ctx, first, who)) || (rc = check_map(ctx, last, who))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
      return set_error(ctx, VGICP_EHIP, std::string(who) + ": hipSetDevice");
    const vgicp_map m[2] = {last, first};
    double mp[24];
    std::memcpy(mp, h_last_pose, 12 * sizeof(double));
    std::memcpy(mp + 12, h_first_pose, 12 * sizeof(double));
    rc = overlap_of_cloud(ctx, *frame, h_pose, m, mp, 2, nullptr, ov, who);
    if (rc) return rc;
  }
  *decision = submap_decision(*rules, n_submap, ov[0], ov[1]);
  if (overlap_last) *overlap_last = ov[0];
  if (overlap_first) *overlap_first = ov[1];
  return VGICP_OK;
}

// ------------------------------------------------------------------ server

int vgicp_server_connect(vgicp_server srv, int32_t frame, const double *h_pose,
                         const int32_t *candidates, const double *h_candidate_poses,
                         int32_t n_candidates, double threshold, int32_t rule, int64_t *h_hits,
                         double *h_overlap, int32_t *h_admitted, int32_t *n_admitted) {
  if (!srv) return VGICP_EINVAL;
  if (n_candidates < 0 || (n_candidates > 0 && (!candidates || !h_candidate_poses || !h_admitted)) ||
      !h_pose || !std::isfinite(threshold) ||
      (rule != VGICP_GATE_ABOVE && rule != VGICP_GATE_AT_LEAST))
    return VGICP_EINVAL;
  const int64_t max_poses = server_max_batch_poses(srv);
  if (max_poses < 2) return VGICP_EINVAL;
  // one overlap request per chunk of candidates (each carries the frame's pose
  // and the chunk's poses), all in flight before the first wait
  const int64_t per = max_poses - 1;
  std::vector<int64_t> hits(size_t(std::max(n_candidates, 1)));
  std::vector<double> ov(size_t(std::max(n_candidates, 1)));
  std::vector<int64_t> tickets;
  int rc = VGICP_OK;
  for (int64_t b = 0; b < n_candidates && rc == VGICP_OK; b += per) {
    const int64_t cnt = std::min<int64_t>(per, n_candidates - b);
    std::vector<vgicp_factor> rows(static_cast<size_t>(cnt));
    std::vector<double> poses(static_cast<size_t>(cnt + 1) * 12);
    std::memcpy(poses.data(), h_pose, 12 * sizeof(double));
    for (int64_t k = 0; k < cnt; ++k) {
      rows[size_t(k)] = vgicp_factor{frame, candidates[b + k], 0, int32_t(k + 1)};
      std::memcpy(poses.data() + 12 * (k + 1), h_candidate_poses + 12 * (b + k),
                  12 * sizeof(double));
    }
    int64_t ticket = 0;
    rc = vgicp_server_submit(srv, VGICP_REQ_OVERLAP, rows.data(), cnt, poses.data(),
                             int32_t(cnt + 1), nullptr, nullptr, nullptr, hits.data() + b,
                             ov.data() + b, &ticket);
    if (rc == VGICP_OK) tickets.push_back(ticket);
  }
  for (int64_t tk : tickets) {
    const int wrc = vgicp_server_wait(srv, tk, nullptr);
    if (rc == VGICP_OK) rc = wrc;
  }
  if (rc != VGICP_OK) return rc;
  int32_t count = 0;
  for (int32_t k = 0; k < n_candidates; ++k) {
    h_admitted[k] = admitted_by(ov[size_t(k)], threshold, rule) ? 1 : 0;
    count += h_admitted[k];
    if (h_hits) h_hits[k] = hits[size_t(k)];
    if (h_overlap) h_overlap[k] = ov[size_t(k)];
  }
  if (n_admitted) *n_admitted = count;
  return VGICP_OK;
}

int vgicp_server_submap_step(vgicp_server srv, const vgicp_submap_rules *rules, int32_t frame,
                             const double *h_pose, int32_t first, const double *h_first_pose,
                             int32_t last, const double *h_last_pose, int32_t n_submap,
                             int32_t *decision, double *overlap_first, double *overlap_last) {
  if (!srv) return VGICP_EINVAL;
  std::string msg;
  if (check_rules(rules, msg) || !decision || n_submap < 0) return VGICP_EINVAL;
  double ov[2] = {0.0, 0.0};  // last, first
  if (n_submap > 0) {
    if (!h_pose || !h_first_pose || !h_last_pose) return VGICP_EINVAL;
    const vgicp_factor rows[2] = {{frame, last, 0, 1}, {frame, first, 0, 2}};
    double poses[36];
    std::memcpy(poses, h_pose, 12 * sizeof(double));
    std::memcpy(poses + 12, h_last_pose, 12 * sizeof(double));
    std::memcpy(poses + 24, h_first_pose, 12 * sizeof(double));
    int64_t hits[2] = {0, 0};
    int64_t ticket = 0;
    int rc = vgicp_server_submit(srv, VGICP_REQ_OVERLAP, rows, 2, poses, 3, nullptr, nullptr,
                                 nullptr, hits, ov, &ticket);
    if (rc == VGICP_OK) rc = vgicp_server_wait(srv, ticket, nullptr);
    if (rc != VGICP_OK) return rc;
  }
  *decision = submap_decision(*rules, n_submap, ov[0], ov[1]);
  if (overlap_last) *overlap_last = ov[0];
  if (overlap_first) *overlap_first = ov[1];
  return VGICP_OK;
}

}  // extern "C"
