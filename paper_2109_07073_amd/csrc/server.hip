// Continuous-batching server over resident keyframes (vgicp_server_* in
// include/vgicp.h).
//
// One worker thread owns `inflight` batch slots, each with its own stream,
// device tables and pinned staging.  Requests are queued by vgicp_server_submit;
// the worker packs queued requests of one kind, FIFO, into the next free slot
// (splitting a request across batches when it does not fit), uploads the
// slot's factor/tile/pose tables, launches the same kernels as the factor-set
// path and copies the outputs back.  A host function enqueued after each batch
// wakes the worker, which scatters the outputs into the requests' buffers.
// New requests are admitted while earlier batches are still running.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "vgicp_internal.hpp"

namespace vgicp {
int voxelize_impl(vgicp_ctx ctx, const vgicp_cloud *cloud, double resolution, vgicp_map *out,
                  std::string &msg);
hipError_t launch_linearize(const vgicp_factorset_s *fs, int accum, int resid, int fused,
                            float kappa,
                            bool lin, int64_t tb, int64_t te, const double *poses, int32_t *corr,
                            hipStream_t st, int32_t stride = 1, const void *consts = nullptr);
hipError_t launch_overlap(const vgicp_factorset_s *fs, int64_t tb, int64_t te,
                          const double *poses, hipStream_t st, int32_t stride = 1);
hipError_t launch_reduce(const vgicp_factorset_s *fs, int64_t f0, int64_t nf, const double *poses,
                         int mode, double *H, double *b, double *e, int64_t *inl,
                         double *overlap, hipStream_t st);
}  // namespace vgicp

using namespace vgicp;
using Clock = std::chrono::steady_clock;

namespace {


struct Frame {
  bool live = false;
  // device: xyz (the caller's [3][n] while the frame is voxelized, then its
  // ordered copy [n][3]), then cov [n][6] at cov_offset floats
  float *cloud = nullptr;
  int64_t cov_offset = 0;  // 3n rounded up to a multiple of 4 floats (16 bytes)
  int64_t n = 0;
  vgicp_map map = nullptr;
  int64_t bytes = 0;
  int64_t users = 0;       // factors of queued or running requests that read it
  bool remove_pending = false;
};

struct Request {
  int64_t ticket = 0;
  int kind = 0;
  std::vector<vgicp_factor> factors;
  std::vector<double> poses;  // [n_poses][12]
  double *H = nullptr, *b = nullptr, *e = nullptr, *overlap = nullptr;
  int64_t *inliers = nullptr;
  int64_t next = 0;       // first factor not yet put in a batch
  int64_t remaining = 0;  // factors whose outputs are not written yet
  Clock::time_point t_submit;
  double latency_ms = 0.0;
  bool done = false;
  bool failed = false;
};

// A contiguous run of one request's factors inside a batch.
struct Chunk {
  std::shared_ptr<Request> req;
  int64_t first;      // factor index in the request
  int64_t count;
  int64_t batch_pos;  // position of the first factor in the batch
};

// A batch moves its inputs to the device with one copy and its outputs back
// with one: the inputs packed as [descriptors | tiles | poses] (each part
// 256-byte aligned), the outputs of nf factors as [inliers | e | overlap | b |
// H] (nf, nf, nf, 12 nf and 144 nf eight-byte values).
constexpr size_t kOutPerFactor = 159;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Slot {
  hipStream_t stream = nullptr;
  // device
  unsigned char *d_in = nullptr;
  double *d_out = nullptr;
  double *d_partials = nullptr;
  // pinned host staging: the descriptors are written in place in h_in, tiles
  // and poses gathered there at launch
  unsigned char *h_in = nullptr;
  double *h_out = nullptr;
  FactorDesc *h_factors = nullptr;  // = h_in
  Tile *h_tiles = nullptr;
  double *h_poses = nullptr;
  // batch in flight
  bool busy = false;
  bool finished = false;
  hipError_t err = hipSuccess;
  int kind = 0;
  int64_t n_factors = 0;
  std::vector<Chunk> chunks;
  std::vector<int32_t> frames_used;  // one entry per factor (source and target)
  uint64_t seq = 0;
};

}  // namespace

struct vgicp_server_s {
  int device = 0;
  vgicp_server_config cfg{};
  int tile_points = kDefaultTile;
  int64_t max_tiles = 0;
  vgicp_context_s ingest;  // stream + scratch for voxelization
  std::mutex mu;
  std::condition_variable cv;       // worker wake-up
  std::condition_variable done_cv;  // request completion
  std::deque<std::shared_ptr<Request>> pending;
  std::unordered_map<int64_t, std::shared_ptr<Request>> requests;
  std::vector<Frame> frames;
  std::vector<Slot> slots;
  int64_t used_bytes = 0;
  int64_t next_ticket = 1;
  uint64_t batch_seq = 0;
  bool stop = false;
  std::thread worker;
  std::mutex ingest_mu;  // one voxelization at a time (the ingest scratch is shared)
  std::string last_error;
  std::mutex err_mu;
  int64_t callbacks_outstanding = 0;  // completion callbacks enqueued and not yet run
  // stats
  int64_t n_batches = 0, n_completed = 0, max_req_per_batch = 0, max_inflight = 0;
};

namespace {

int srv_fail(vgicp_server s, int code, const std::string &msg) {
  if (s) {
    std::lock_guard<std::mutex> g(s->err_mu);
    s->last_error = msg;
  }
  return code;
}

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
  return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(1, count) * sizeof(T));
}
template <typename T>
hipError_t host_alloc(T **p, size_t count) {
  return hipHostMalloc(reinterpret_cast<void **>(p), std::max<size_t>(1, count) * sizeof(T),
                       hipHostMallocDefault);
}

void free_slot(Slot &s) {
  if (s.stream) (void)hipStreamDestroy(s.stream);
  for (void *p : {(void *)s.d_in, (void *)s.d_out, (void *)s.d_partials})
    if (p) (void)hipFree(p);
  for (void *p : {(void *)s.h_in, (void *)s.h_out, (void *)s.h_tiles, (void *)s.h_poses})
    if (p) (void)hipHostFree(p);
}

// Bytes of a packed input block for F descriptors, T tiles and P poses.
size_t in_block_bytes(int64_t F, int64_t T, int64_t P) {
  return align256(size_t(F) * sizeof(FactorDesc)) + align256(size_t(T) * sizeof(Tile)) +
         size_t(P) * 12 * sizeof(double);
}

hipError_t alloc_slot(Slot &s, int64_t F, int64_t T, int64_t P) {
  hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
  const size_t in_bytes = in_block_bytes(F, T, P);
  if (e == hipSuccess) e = dev_alloc(&s.d_in, in_bytes);
  if (e == hipSuccess) e = dev_alloc(&s.d_out, size_t(F) * kOutPerFactor);
  if (e == hipSuccess) e = dev_alloc(&s.d_partials, T * kPartialStride);
  if (e == hipSuccess) e = host_alloc(&s.h_in, in_bytes);
  if (e == hipSuccess) e = host_alloc(&s.h_out, size_t(F) * kOutPerFactor);
  if (e == hipSuccess) e = host_alloc(&s.h_tiles, T);
  if (e == hipSuccess) e = host_alloc(&s.h_poses, P * 12);
  s.h_factors = reinterpret_cast<FactorDesc *>(s.h_in);
  return e;
}

struct DoneArgs {
  vgicp_server srv;
  size_t slot;
};

// Runs on the HIP runtime's callback thread.  Everything it does to the
// server happens under the lock, and the server is destroyed only once no
// callback is outstanding, so it never touches a freed server.
void on_batch_done(void *p) {
  DoneArgs *a = static_cast<DoneArgs *>(p);
  vgicp_server srv = a->srv;
  const size_t slot = a->slot;
  delete a;
  std::lock_guard<std::mutex> g(srv->mu);
  srv->slots[slot].finished = true;
  srv->callbacks_outstanding -= 1;
  srv->cv.notify_all();
}

int64_t request_points(const vgicp_server_s *srv, const vgicp_factor &f) {
  return srv->frames[size_t(f.src)].n;
}

// Drop the frame references of a request that will not run.
void release_frames_of(vgicp_server srv, const Request &r) {
  for (int64_t k = r.next; k < int64_t(r.factors.size()); ++k) {
    srv->frames[size_t(r.factors[size_t(k)].src)].users -= 1;
    srv->frames[size_t(r.factors[size_t(k)].tgt)].users -= 1;
  }
}

// Pack queued requests of the kind at the head of the queue into slot `si`
// and launch it.  Called with the lock held.
void launch_batch(vgicp_server srv, size_t si) {
  Slot &s = srv->slots[si];
  s.chunks.clear();
  s.frames_used.clear();
  const int kind = srv->pending.front()->kind;
  const int64_t F = srv->cfg.max_batch_factors;
  const int64_t Pmax = srv->cfg.max_batch_poses;
  const int64_t tp = srv->tile_points;
  int64_t nf = 0, nt = 0, npose = 0, npts = 0;
  while (!srv->pending.empty()) {
    auto req = srv->pending.front();
    if (req->kind != kind) break;
    const int64_t req_poses = int64_t(req->poses.size() / 12);
    if (npose + req_poses > Pmax) break;
    const int64_t pose_base = npose;
    int64_t first = req->next, count = 0;
    while (req->next < int64_t(req->factors.size()) && nf < F) {
      const vgicp_factor &x = req->factors[size_t(req->next)];
      const int64_t n = request_points(srv, x);
      const int64_t tiles = (n + tp - 1) / tp;
      if (nf > 0 && (npts + n > srv->cfg.max_batch_points || nt + tiles > srv->max_tiles)) break;
      FactorDesc &d = s.h_factors[nf];
      std::memset(&d, 0, sizeof(d));
      const Frame &src = srv->frames[size_t(x.src)];
      const Frame &tgt = srv->frames[size_t(x.tgt)];
      d.xyz = src.cloud;
      d.cov = src.cloud + src.cov_offset;
      d.bricks = tgt.map->bricks;
      d.stats = tgt.map->stats;
      d.occ = tgt.map->occ;
      d.occ_mask = occ_bits(tgt.map->capacity) - 1u;
      d.info = tgt.map->info;
      d.n = src.n;
      d.pose_i = int32_t(pose_base + x.pose_i);
      d.pose_j = int32_t(pose_base + x.pose_j);
      d.log2cap = tgt.map->log2cap;
      d.scale = tgt.map->scale;
      d.n_voxels = uint32_t(tgt.map->n_voxels);
      d.tile_begin = int32_t(nt);
      for (int64_t st = 0; st < n; st += tp) s.h_tiles[nt++] = Tile{int32_t(nf), int32_t(st)};
      d.n_tiles = int32_t(nt - d.tile_begin);
      d.tile_stride = 1;
      d.tile_points = int32_t(tp);
      s.frames_used.push_back(x.src);
      s.frames_used.push_back(x.tgt);
      npts += n;
      ++nf;
      ++count;
      ++req->next;
    }
    if (count == 0) break;  // the slot is full
    std::memcpy(s.h_poses + npose * 12, req->poses.data(), req->poses.size() * sizeof(double));
    npose += req_poses;
    s.chunks.push_back(Chunk{req, first, count, nf - count});
    if (req->next == int64_t(req->factors.size())) {
      srv->pending.pop_front();
    } else {
      break;  // the rest of this request goes to the next batch
    }
  }
  if (nf == 0) {  // cannot happen for validated requests; never spin on one
    auto req = srv->pending.front();
    srv->pending.pop_front();
    release_frames_of(srv, *req);
    req->failed = true;
    req->done = true;
    ++srv->n_completed;
    srv->done_cv.notify_all();
    return;
  }
  s.kind = kind;
  s.n_factors = nf;
  s.busy = true;
  s.finished = false;
  s.err = hipSuccess;
  s.seq = ++srv->batch_seq;
  ++srv->n_batches;
  srv->max_req_per_batch = std::max<int64_t>(srv->max_req_per_batch, int64_t(s.chunks.size()));
  int64_t inflight = 0;
  for (const Slot &o : srv->slots) inflight += o.busy ? 1 : 0;
  srv->max_inflight = std::max(srv->max_inflight, inflight);

  // one copy in: descriptors (written in place), tiles and poses packed
  const size_t off_tiles = align256(size_t(nf) * sizeof(FactorDesc));
  const size_t off_poses = off_tiles + align256(size_t(nt) * sizeof(Tile));
  const size_t in_bytes = off_poses + size_t(npose) * 12 * sizeof(double);
  std::memcpy(s.h_in + off_tiles, s.h_tiles, size_t(nt) * sizeof(Tile));
  std::memcpy(s.h_in + off_poses, s.h_poses, size_t(npose) * 12 * sizeof(double));
  double *d_poses = reinterpret_cast<double *>(s.d_in + off_poses);
  vgicp_factorset_s view;
  view.device = srv->device;
  view.n_factors = nf;
  view.n_tiles = nt;
  view.tile_points = int32_t(tp);
  view.d_factors = reinterpret_cast<FactorDesc *>(s.d_in);
  view.d_tiles = reinterpret_cast<Tile *>(s.d_in + off_tiles);
  view.d_partials = s.d_partials;
  // outputs [inliers | e | overlap | b | H]
  int64_t *d_inl = reinterpret_cast<int64_t *>(s.d_out);
  double *d_e = s.d_out + nf, *d_ov = s.d_out + 2 * nf;
  double *d_b = s.d_out + 3 * nf, *d_H = s.d_out + 15 * nf;
  const hipStream_t st = s.stream;
  const vgicp_opts &o = srv->cfg.opts;
  hipError_t e = hipMemcpyAsync(s.d_in, s.h_in, in_bytes, hipMemcpyHostToDevice, st);
  size_t out_values = 0;
  if (kind == VGICP_REQ_OVERLAP) {
    if (e == hipSuccess) e = launch_overlap(&view, 0, nt, d_poses, st);
    if (e == hipSuccess)
      e = launch_reduce(&view, 0, nf, d_poses, 2, nullptr, nullptr, nullptr, d_inl, d_ov, st);
    out_values = 3 * size_t(nf);
  } else {
    const bool lin = kind == VGICP_REQ_LINEARIZE;
    if (e == hipSuccess)
      e = launch_linearize(&view, o.accum, o.resid, o.fused, o.fp64_kappa, lin, 0, nt, d_poses,
                           nullptr, st);
    if (e == hipSuccess)
      e = launch_reduce(&view, 0, nf, d_poses, lin ? 0 : 1, d_H, d_b, d_e, d_inl, nullptr, st);
    out_values = (lin ? kOutPerFactor : 2) * size_t(nf);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.h_out, s.d_out, out_values * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) {
    srv->callbacks_outstanding += 1;
    e = hipLaunchHostFunc(st, on_batch_done, new DoneArgs{srv, si});
    if (e != hipSuccess) srv->callbacks_outstanding -= 1;
  }
  if (e != hipSuccess) {
    s.err = e;
    s.finished = true;  // retired as failed by the worker
  }
}

void release_frames(vgicp_server srv, const std::vector<int32_t> &used) {
  for (int32_t f : used) srv->frames[size_t(f)].users -= 1;
}

void free_frame(Frame &fr) {
  if (fr.map) vgicp_map_free(fr.map);
  if (fr.cloud) (void)hipFree(fr.cloud);
  fr = Frame();
}

// Scatter a finished batch into its requests.  Called with the lock held;
// frames whose removal was pending are moved to `to_free` (freed by the caller
// after it drops the lock: the completion callback takes the lock, so no
// blocking HIP call may run under it).
void retire(vgicp_server srv, Slot &s, std::vector<Frame> &to_free) {
  const bool ok = s.err == hipSuccess;
  const int64_t nf = s.n_factors;
  const int64_t *h_inl = reinterpret_cast<const int64_t *>(s.h_out);
  const double *h_e = s.h_out + nf, *h_ov = s.h_out + 2 * nf;
  const double *h_b = s.h_out + 3 * nf, *h_H = s.h_out + 15 * nf;
  for (const Chunk &c : s.chunks) {
    Request &r = *c.req;
    if (ok) {
      for (int64_t k = 0; k < c.count; ++k) {
        const int64_t f = c.first + k, p = c.batch_pos + k;
        if (r.inliers) r.inliers[f] = h_inl[p];
        if (s.kind == VGICP_REQ_OVERLAP) {
          if (r.overlap) r.overlap[f] = h_ov[p];
        } else {
          if (r.e) r.e[f] = h_e[p];
          if (s.kind == VGICP_REQ_LINEARIZE) {
            std::memcpy(r.H + f * 144, h_H + p * 144, 144 * sizeof(double));
            std::memcpy(r.b + f * 12, h_b + p * 12, 12 * sizeof(double));
          }
        }
      }
    } else {
      r.failed = true;
    }
    r.remaining -= c.count;
    if (r.remaining == 0 && !r.done) {
      r.done = true;
      r.latency_ms =
          std::chrono::duration<double, std::milli>(Clock::now() - r.t_submit).count();
      ++srv->n_completed;
    }
  }
  release_frames(srv, s.frames_used);
  for (Frame &fr : srv->frames)
    if (fr.live && fr.remove_pending && fr.users == 0) {
      srv->used_bytes -= fr.bytes;
      to_free.push_back(fr);
      fr = Frame();
    }
  s.chunks.clear();
  s.frames_used.clear();
  s.busy = false;
  s.finished = false;
}

void worker_loop(vgicp_server srv) {
  (void)hipSetDevice(srv->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    bool progressed = false;
    std::vector<Frame> to_free;
    // retire finished batches
    for (Slot &s : srv->slots) {
      if (!s.busy || !s.finished) continue;
      if (s.err == hipSuccess) {
        const hipError_t q = hipStreamQuery(s.stream);
        if (q != hipSuccess && q != hipErrorNotReady) s.err = q;
      }
      retire(srv, s, to_free);
      progressed = true;
    }
    if (progressed) srv->done_cv.notify_all();
    if (!to_free.empty()) {
      lk.unlock();
      for (Frame &fr : to_free) free_frame(fr);
      lk.lock();
    }
    // admit queued requests into free slots
    for (size_t i = 0; i < srv->slots.size() && !srv->pending.empty(); ++i) {
      if (!srv->slots[i].busy) {
        launch_batch(srv, i);
        progressed = true;
      }
    }
    bool any_busy = false;
    for (const Slot &s : srv->slots) any_busy |= s.busy;
    if (srv->stop && srv->pending.empty() && !any_busy) break;
    if (!progressed) srv->cv.wait(lk);
  }
}

std::shared_ptr<Request> find_request(vgicp_server srv, int64_t ticket) {
  auto it = srv->requests.find(ticket);
  return it == srv->requests.end() ? nullptr : it->second;
}

}  // namespace

int64_t vgicp::server_max_batch_poses(vgicp_server srv) { return srv->cfg.max_batch_poses; }

extern "C" {

int vgicp_server_create(int device, const vgicp_server_config *cfg, vgicp_server *out) {
  if (!out || !cfg) return VGICP_EINVAL;
  *out = nullptr;
  if (cfg->max_batch_factors < 1 || cfg->max_batch_points < 1 || cfg->max_batch_poses < 1 ||
      cfg->inflight < 1 || cfg->inflight > 8 || cfg->memory_budget_bytes < 0 ||
      cfg->reserved != 0)
    return VGICP_EINVAL;
  int tp = cfg->tile_points ? cfg->tile_points : kDefaultTile;
  if (tp < 256 || tp > (1 << 20) || tp % 256 != 0) return VGICP_EINVAL;
  const vgicp_opts &o = cfg->opts;
  if ((o.accum != VGICP_ACC_MIXED && o.accum != VGICP_ACC_F32 && o.accum != VGICP_ACC_F64 &&
       o.accum != VGICP_ACC_F32_COMP) ||
      (o.resid != VGICP_RESID_F64 && o.resid != VGICP_RESID_F32) || !(o.fp64_kappa >= 0.0f) ||
      !std::isfinite(o.fp64_kappa) || (o.fused != VGICP_FUSED_F64 && o.fused != VGICP_FUSED_F32) ||
      (o.form != VGICP_FORM_AUTO && o.form != VGICP_FORM_SOURCE))
    return VGICP_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VGICP_EHIP;
  if (hipSetDevice(device) != hipSuccess) return VGICP_EHIP;
  auto *srv = new (std::nothrow) vgicp_server_s();
  if (!srv) return VGICP_ENOMEM;
  srv->device = device;
  srv->cfg = *cfg;
  srv->tile_points = tp;
  srv->max_tiles = (int64_t(cfg->max_batch_points) + tp - 1) / tp + cfg->max_batch_factors;
  srv->ingest.device = device;
  hipError_t e = hipStreamCreateWithFlags(&srv->ingest.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&srv->ingest.err_word, 256);
  if (e == hipSuccess) e = hipHostMalloc(&srv->ingest.host_pinned, 64, hipHostMallocDefault);
  srv->slots.resize(size_t(cfg->inflight));
  for (Slot &s : srv->slots)
    if (e == hipSuccess) e = alloc_slot(s, cfg->max_batch_factors, srv->max_tiles,
                                        cfg->max_batch_poses);
  if (e != hipSuccess) {
    for (Slot &s : srv->slots) free_slot(s);
    if (srv->ingest.stream) (void)hipStreamDestroy(srv->ingest.stream);
    if (srv->ingest.err_word) (void)hipFree(srv->ingest.err_word);
    if (srv->ingest.host_pinned) (void)hipHostFree(srv->ingest.host_pinned);
    delete srv;
    return e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP;
  }
  srv->worker = std::thread(worker_loop, srv);
  *out = srv;
  return VGICP_OK;
}

int vgicp_server_destroy(vgicp_server srv) {
  if (!srv) return VGICP_OK;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv.wait(lk, [&] { return srv->callbacks_outstanding == 0; });
  }
  (void)hipSetDevice(srv->device);
  for (Slot &s : srv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot(s);
  }
  for (Frame &fr : srv->frames)
    if (fr.live) free_frame(fr);
  if (srv->ingest.stream) (void)hipStreamSynchronize(srv->ingest.stream);
  if (srv->ingest.scratch) (void)hipFree(srv->ingest.scratch);
  if (srv->ingest.stream) (void)hipStreamDestroy(srv->ingest.stream);
  if (srv->ingest.err_word) (void)hipFree(srv->ingest.err_word);
  if (srv->ingest.host_pinned) (void)hipHostFree(srv->ingest.host_pinned);
  delete srv;
  return VGICP_OK;
}

const char *vgicp_server_last_error(vgicp_server srv) {
  static const char *none = "";
  if (!srv) return "vgicp_server_last_error: server is NULL";
  std::lock_guard<std::mutex> g(srv->err_mu);
  return srv->last_error.empty() ? none : srv->last_error.c_str();
}

int vgicp_server_add_frame(vgicp_server srv, const float *h_xyz, const float *h_cov, int64_t n,
                           double resolution, int32_t *frame_id) {
  if (!srv) return VGICP_EINVAL;
  if (!frame_id) return srv_fail(srv, VGICP_EINVAL, "vgicp_server_add_frame: frame_id is NULL");
  if (n < 0 || n > kMaxCloudPoints || (n > 0 && (!h_xyz || !h_cov)))
    return srv_fail(srv, VGICP_EINVAL, "vgicp_server_add_frame: bad cloud");
  if (!std::isfinite(resolution) || !(resolution > 0.0))
    return srv_fail(srv, VGICP_EINVAL, "vgicp_server_add_frame: bad resolution");
  if (hipSetDevice(srv->device) != hipSuccess)
    return srv_fail(srv, VGICP_EHIP, "vgicp_server_add_frame: hipSetDevice");
  Frame fr;
  fr.n = n;
  fr.cov_offset = (3 * n + 3) & ~int64_t(3);
  const size_t cloud_bytes =
      size_t(std::max<int64_t>(fr.cov_offset + 6 * n, 1)) * sizeof(float);
  hipError_t e = hipMalloc(&fr.cloud, cloud_bytes);
  if (e == hipSuccess && n > 0)
    e = hipMemcpy(fr.cloud, h_xyz, size_t(3 * n) * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess && n > 0)
    e = hipMemcpy(fr.cloud + fr.cov_offset, h_cov, size_t(6 * n) * sizeof(float),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (fr.cloud) (void)hipFree(fr.cloud);
    return srv_fail(srv, e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP,
                    std::string("vgicp_server_add_frame: ") + hipGetErrorString(e));
  }
  vgicp_cloud c{fr.cloud, fr.cloud + fr.cov_offset, n};
  std::string msg;
  int rc;
  {
    std::lock_guard<std::mutex> g(srv->ingest_mu);
    rc = voxelize_impl(&srv->ingest, &c, resolution, &fr.map, msg);
    if (rc == VGICP_OK && hipStreamSynchronize(srv->ingest.stream) != hipSuccess) {
      rc = VGICP_EHIP;
      msg = "vgicp_server_add_frame: voxelization failed";
    }
    // Then the frame's points are put in Morton order of cells of its own
    // resolution (the order a factor set gives a cloud matched against maps of
    // that resolution), so that its rounds read neighbouring voxels together,
    // and its coordinates are kept point by point, as the kernels read them.
    // Requests have no per-point outputs, so the permutation is not kept.
    if (rc == VGICP_OK && n > 0) {
      const std::vector<double> cell{resolution};
      std::vector<SortedSource> ss;
      void *buf = nullptr;
      hipStream_t st = srv->ingest.stream;
      hipError_t se = make_sorted_sources(&c, 1, cell, &buf, ss, st);
      if (se == hipSuccess && buf) {
        se = hipMemcpyAsync(fr.cloud, ss[0].xyz, size_t(3 * n) * sizeof(float),
                            hipMemcpyDeviceToDevice, st);
        if (se == hipSuccess)
          se = hipMemcpyAsync(fr.cloud + fr.cov_offset, ss[0].cov, size_t(6 * n) * sizeof(float),
                              hipMemcpyDeviceToDevice, st);
        const hipError_t ye = hipStreamSynchronize(st);
        if (se == hipSuccess) se = ye;
      }
      if (buf) (void)hipFree(buf);
      if (se != hipSuccess) {
        vgicp_map_free(fr.map);
        fr.map = nullptr;
        rc = se == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP;
        msg = std::string("vgicp_server_add_frame: ") + hipGetErrorString(se);
      }
    }
  }
  if (rc != VGICP_OK) {
    (void)hipFree(fr.cloud);
    return srv_fail(srv, rc, msg);
  }
  fr.bytes = int64_t(cloud_bytes) + fr.map->device_bytes();
  fr.live = true;
  std::unique_lock<std::mutex> g(srv->mu);
  if (srv->cfg.memory_budget_bytes > 0 && srv->used_bytes + fr.bytes > srv->cfg.memory_budget_bytes) {
    g.unlock();
    free_frame(fr);
    return srv_fail(srv, VGICP_EFULL, "vgicp_server_add_frame: memory budget exceeded");
  }
  srv->used_bytes += fr.bytes;
  int32_t id = -1;
  for (size_t i = 0; i < srv->frames.size(); ++i)
    if (!srv->frames[i].live) {
      id = int32_t(i);
      break;
    }
  if (id < 0) {
    id = int32_t(srv->frames.size());
    srv->frames.emplace_back();
  }
  srv->frames[size_t(id)] = fr;
  *frame_id = id;
  return VGICP_OK;
}

int vgicp_server_remove_frame(vgicp_server srv, int32_t frame_id) {
  if (!srv) return VGICP_EINVAL;
  Frame gone;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (frame_id < 0 || size_t(frame_id) >= srv->frames.size() ||
        !srv->frames[size_t(frame_id)].live || srv->frames[size_t(frame_id)].remove_pending)
      return srv_fail(srv, VGICP_EINVAL, "vgicp_server_remove_frame: unknown frame");
    Frame &fr = srv->frames[size_t(frame_id)];
    if (fr.users > 0) {
      fr.remove_pending = true;  // freed when its last request retires
      return VGICP_OK;
    }
    srv->used_bytes -= fr.bytes;
    gone = fr;
    fr = Frame();
  }
  (void)hipSetDevice(srv->device);
  free_frame(gone);
  return VGICP_OK;
}

int vgicp_server_memory(vgicp_server srv, int64_t *used_bytes, int64_t *budget_bytes) {
  if (!srv) return VGICP_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  if (used_bytes) *used_bytes = srv->used_bytes;
  if (budget_bytes) *budget_bytes = srv->cfg.memory_budget_bytes;
  return VGICP_OK;
}

int vgicp_server_submit(vgicp_server srv, int kind, const vgicp_factor *factors, int64_t n,
                        const double *h_poses, int32_t n_poses, double *H, double *b, double *e,
                        int64_t *inliers, double *overlap, int64_t *ticket) {
  const vgicp_server_request r{kind, n_poses, n, factors, h_poses, H, b, e, inliers, overlap};
  return vgicp_server_submit_many(srv, &r, 1, ticket);
}

int vgicp_server_submit_many(vgicp_server srv, const vgicp_server_request *reqs, int32_t n_reqs,
                             int64_t *tickets) {
  if (!srv) return VGICP_EINVAL;
  const char *who = n_reqs == 1 ? "vgicp_server_submit" : "vgicp_server_submit_many";
  if (n_reqs < 0 || (n_reqs > 0 && (!reqs || !tickets)))
    return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": bad request or ticket array");
  // every argument checked and copied before anything is queued
  std::vector<std::shared_ptr<Request>> batch;
  batch.reserve(size_t(n_reqs));
  for (int32_t q = 0; q < n_reqs; ++q) {
    const vgicp_server_request &r = reqs[q];
    if (r.kind < VGICP_REQ_LINEARIZE || r.kind > VGICP_REQ_OVERLAP)
      return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": unknown kind");
    if (r.n < 0 || (r.n > 0 && !r.factors) || r.n_poses < 0 || (r.n_poses > 0 && !r.h_poses))
      return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": bad factor or pose arrays");
    if (r.n_poses > srv->cfg.max_batch_poses)
      return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": more poses than max_batch_poses");
    if (r.n > 0 && !r.inliers) return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": inliers is NULL");
    if (r.n > 0 && r.kind == VGICP_REQ_LINEARIZE && (!r.H || !r.b || !r.e))
      return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": H, b or e is NULL");
    if (r.n > 0 && r.kind == VGICP_REQ_EVALUATE && !r.e)
      return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": e is NULL");
    for (int64_t k = 0; k < int64_t(r.n_poses) * 12; ++k)
      if (!std::isfinite(r.h_poses[k]))
        return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": non-finite pose");
    auto req = std::make_shared<Request>();
    req->kind = r.kind;
    req->factors.assign(r.factors, r.factors + r.n);
    req->poses.assign(r.h_poses, r.h_poses + size_t(r.n_poses) * 12);
    req->H = r.H;
    req->b = r.b;
    req->e = r.e;
    req->inliers = r.inliers;
    req->overlap = r.overlap;
    req->remaining = r.n;
    batch.push_back(std::move(req));
  }
  const auto now = Clock::now();
  {
    std::lock_guard<std::mutex> g(srv->mu);
    auto bad_frame = [&](int32_t f) {
      return f < 0 || size_t(f) >= srv->frames.size() || !srv->frames[size_t(f)].live ||
             srv->frames[size_t(f)].remove_pending;
    };
    for (size_t q = 0; q < batch.size(); ++q) {
      const int32_t n_poses = reqs[q].n_poses;
      for (const vgicp_factor &x : batch[q]->factors) {
        if (bad_frame(x.src) || bad_frame(x.tgt) || x.pose_i < 0 || x.pose_i >= n_poses ||
            x.pose_j < 0 || x.pose_j >= n_poses)
          return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": factor references an unknown "
                                                                "frame or pose");
        if (srv->frames[size_t(x.src)].n > srv->cfg.max_batch_points)
          return srv_fail(srv, VGICP_EINVAL, std::string(who) + ": a source frame has more "
                                                                "points than max_batch_points");
      }
    }
    for (size_t q = 0; q < batch.size(); ++q) {
      Request &req = *batch[q];
      for (const vgicp_factor &x : req.factors) {
        srv->frames[size_t(x.src)].users += 1;
        srv->frames[size_t(x.tgt)].users += 1;
      }
      req.t_submit = now;
      req.ticket = srv->next_ticket++;
      tickets[q] = req.ticket;
      srv->requests[req.ticket] = batch[q];
      if (req.factors.empty()) {
        req.done = true;
        ++srv->n_completed;
      } else {
        srv->pending.push_back(batch[q]);
      }
    }
  }
  srv->cv.notify_all();
  return VGICP_OK;
}

int vgicp_server_poll(vgicp_server srv, int64_t ticket, int *done) {
  if (!srv || !done) return VGICP_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  auto r = find_request(srv, ticket);
  if (!r) return srv_fail(srv, VGICP_EINVAL, "vgicp_server_poll: unknown ticket");
  *done = r->done ? 1 : 0;
  return VGICP_OK;
}

int vgicp_server_wait(vgicp_server srv, int64_t ticket, double *latency_ms) {
  if (!srv) return VGICP_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto r = find_request(srv, ticket);
  if (!r) return srv_fail(srv, VGICP_EINVAL, "vgicp_server_wait: unknown ticket");
  srv->done_cv.wait(lk, [&] { return r->done; });
  if (latency_ms) *latency_ms = r->latency_ms;
  const bool failed = r->failed;
  srv->requests.erase(ticket);
  if (failed) return srv_fail(srv, VGICP_EHIP, "vgicp_server_wait: a batch of the request failed");
  return VGICP_OK;
}

int vgicp_server_stats(vgicp_server srv, int64_t *batches, int64_t *requests,
                       int64_t *max_requests_per_batch, int64_t *max_inflight) {
  if (!srv) return VGICP_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  if (batches) *batches = srv->n_batches;
  if (requests) *requests = srv->n_completed;
  if (max_requests_per_batch) *max_requests_per_batch = srv->max_req_per_batch;
  if (max_inflight) *max_inflight = srv->max_inflight;
  return VGICP_OK;
}

}  // extern "C"
