// Voxel-map construction on gfx950 (Sec. III-A, VGICP voxel data association).
//
// Each voxel carries the mean of its points and the mean of their
// covariances (the VGICP aggregation of point distributions), accumulated in
// FP64 in point order and rounded once to FP32.  Voxels are stored densely,
// brick after brick (bricks of 4 x 4 x 4 voxels), and found through an
// open-addressed table of brick records holding each brick's occupancy mask.
//
// Steps: keys -> radix sort of (key, point index) -> segment heads -> scan ->
// segment starts -> [host sync: voxel count] -> per voxel its brick-major
// sort key -> radix sort of (brick key and bit, voxel ordinal) -> brick heads
// -> scan -> brick starts -> [host sync: brick count] -> brick table insertion
// and FP64 voxel sums.  This runs once per cloud, off the per-iteration path.

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "vgicp_internal.hpp"

namespace vgicp {

__global__ void __launch_bounds__(256)
k_voxel_keys(const float *__restrict__ xyz, int64_t n, float s, uint64_t *__restrict__ keys,
             uint32_t *__restrict__ idx, uint32_t *__restrict__ err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t bad = 0;
  int32_t k[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = xyz[a * n + i];
    const float v = x * s;
    if (!isfinite(x)) {
      bad |= kErrNonFinite;
      k[a] = 0;
    } else if (!(v >= -kKeyLimitF && v < kKeyLimitF)) {
      bad |= kErrRange;
      k[a] = 0;
    } else {
      k[a] = int32_t(floorf(v));
    }
  }
  if (bad) atomicOr(err, bad);
  keys[i] = pack_key(k[0], k[1], k[2]);
  idx[i] = uint32_t(i);
}

__global__ void __launch_bounds__(256)
k_segment_heads(const uint64_t *__restrict__ sorted_keys, int64_t n, uint32_t *__restrict__ head) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = (i == 0 || sorted_keys[i] != sorted_keys[i - 1]) ? 1u : 0u;
}

// ord1[i] is the inclusive scan of head: the 1-based ordinal of element i.
__global__ void __launch_bounds__(256)
k_segment_starts(const uint32_t *__restrict__ head, const uint32_t *__restrict__ ord1, int64_t n,
                 uint32_t *__restrict__ seg) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (head[i]) seg[ord1[i] - 1] = uint32_t(i);
  if (i == n - 1) seg[ord1[i]] = uint32_t(n);
}

__global__ void __launch_bounds__(256)
k_fill_empty(BrickRecord *__restrict__ bricks, int64_t cap, uint32_t *__restrict__ occ,
             uint32_t occ_words) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < cap) {
    BrickRecord r;
    r.key = kEmptyKey;
    r.mask = 0;
    r.base = 0;
    r.pad[0] = r.pad[1] = r.pad[2] = 0;
    bricks[i] = r;
  }
  if (i < int64_t(occ_words)) occ[i] = 0u;
}

// Per voxel (in lexicographic order): its packed key and its brick-major sort
// key (brick key above the 6-bit position in the brick).
__global__ void __launch_bounds__(256)
k_brick_sortkeys(const uint64_t *__restrict__ sorted_keys, const uint32_t *__restrict__ seg,
                 int64_t n_voxels, uint64_t *__restrict__ vkey, uint64_t *__restrict__ bsort,
                 uint32_t *__restrict__ vord) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n_voxels) return;
  const uint64_t key = sorted_keys[seg[v]];
  const int32_t kx = key_field(key, 0), ky = key_field(key, 1), kz = key_field(key, 2);
  vkey[v] = key;
  bsort[v] = brick_sort_key(kx, ky, kz);
  vord[v] = uint32_t(v);
}

__global__ void __launch_bounds__(256)
k_brick_heads(const uint64_t *__restrict__ bsort, int64_t n_voxels, uint32_t *__restrict__ head) {
  const int64_t d = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (d >= n_voxels) return;
  head[d] = (d == 0 || (bsort[d] >> 6) != (bsort[d - 1] >> 6)) ? 1u : 0u;
}

// One thread per brick: its occupancy mask from its voxels' bits, then
// linear-probing insertion of the record.
__global__ void __launch_bounds__(256)
k_build_bricks(const uint64_t *__restrict__ bsort, const uint32_t *__restrict__ bstart,
               int64_t n_bricks, int64_t n_voxels, BrickRecord *__restrict__ bricks,
               uint32_t log2cap, uint32_t *__restrict__ occ, uint32_t occ_mask) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= n_bricks) return;
  const uint32_t d0 = bstart[b];
  const uint32_t d1 = (b + 1 < n_bricks) ? bstart[b + 1] : uint32_t(n_voxels);
  uint64_t mask = 0;
  for (uint32_t d = d0; d < d1; ++d) mask |= 1ull << (bsort[d] & 63u);
  const uint64_t key = brick_key_of_sort_key(bsort[d0]);
  const uint32_t cmask = (1u << log2cap) - 1u;
  uint32_t h = brick_slot_of_key(key, log2cap);
  // the records of one position in the lines: cap / kProbeStep of them
  for (uint32_t probe = 0; probe <= (cmask >> 2); ++probe) {
    const unsigned long long prev =
        atomicCAS(reinterpret_cast<unsigned long long *>(&bricks[h].key),
                  (unsigned long long)kEmptyKey, (unsigned long long)key);
    if (prev == kEmptyKey) break;
    h = (h + kProbeStep) & cmask;
  }
  bricks[h].mask = mask;
  bricks[h].base = d0;
  const uint32_t bit = h & occ_mask;
  atomicOr(&occ[bit >> 5], 1u << (bit & 31u));
}

// One thread per voxel, by dense (brick-major) position d: sequential FP64
// sums over the voxel's points in point order, one FP64 division, one
// rounding to FP32.
__global__ void __launch_bounds__(256)
k_build_payload(const float *__restrict__ xyz, const float *__restrict__ cov, int64_t n,
                const uint32_t *__restrict__ sorted_idx, const uint32_t *__restrict__ seg,
                const uint32_t *__restrict__ vord, const uint64_t *__restrict__ vkey,
                int64_t n_voxels, VoxelStats *__restrict__ stats,
                VoxelInfo *__restrict__ info) {
  const int64_t d = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (d >= n_voxels) return;
  const uint32_t v = vord[d];
  const uint32_t b = seg[v], e = seg[v + 1];
  double sm[3] = {0.0, 0.0, 0.0};
  double sc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (uint32_t j = b; j < e; ++j) {
    const uint32_t p = sorted_idx[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) sm[a] += double(xyz[a * n + p]);
#pragma unroll
    for (int a = 0; a < 6; ++a) sc[a] += double(cov[6 * int64_t(p) + a]);
  }
  const double cnt = double(e - b);
  VoxelStats st;
#pragma unroll
  for (int a = 0; a < 3; ++a) st.mean[a] = float(sm[a] / cnt);
#pragma unroll
  for (int a = 0; a < 6; ++a) st.cov[a] = float(sc[a] / cnt);
  stats[d] = st;
  VoxelInfo in;
  in.key = vkey[v];
  in.ordinal = int32_t(v);
  in.count = int32_t(e - b);
  info[d] = in;
}

__global__ void __launch_bounds__(256)
k_export(const VoxelStats *__restrict__ stats, const VoxelInfo *__restrict__ info,
         int64_t n_voxels, int32_t *__restrict__ keys, float *__restrict__ mean,
         float *__restrict__ cov, int32_t *__restrict__ count) {
  const int64_t d = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (d >= n_voxels) return;
  const VoxelStats s = stats[d];
  const VoxelInfo in = info[d];
  const int64_t o = in.ordinal;
  if (keys) {
#pragma unroll
    for (int a = 0; a < 3; ++a) keys[3 * o + a] = key_field(in.key, a);
  }
  if (mean) {
#pragma unroll
    for (int a = 0; a < 3; ++a) mean[3 * o + a] = s.mean[a];
  }
  if (cov) {
#pragma unroll
    for (int a = 0; a < 6; ++a) cov[6 * o + a] = s.cov[a];
  }
  if (count) count[o] = in.count;
}

static inline unsigned grid_for(int64_t n, int block = 256) {
  return unsigned((n + block - 1) / block);
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch layout for n points; returns total bytes (rocPRIM temp included).
// After the point sort, keys_in, idx_in, head, ord1 and spare are reused for
// the per-voxel arrays (V <= n): vkey, vord_in, bhead, bord1, vord_out;
// bsort_in/out hold the brick-major sort keys and bstart the brick starts.
struct VoxScratch {
  uint64_t *keys_in, *keys_out, *bsort_in, *bsort_out;
  uint32_t *idx_in, *idx_out, *head, *ord1, *spare, *seg, *bstart;
  void *temp;
  size_t temp_bytes;
};

static hipError_t plan_scratch(int64_t n, hipStream_t stream, size_t *total, size_t *sort_bytes,
                               size_t *scan_bytes) {
  size_t sb = 0, cb = 0;
  hipError_t err = rocprim::radix_sort_pairs(nullptr, sb, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (uint32_t *)nullptr, (uint32_t *)nullptr, size_t(n), 0,
                                             63, stream);
  if (err != hipSuccess) return err;
  err = rocprim::inclusive_scan(nullptr, cb, (uint32_t *)nullptr, (uint32_t *)nullptr, size_t(n),
                                rocprim::plus<uint32_t>(), stream);
  if (err != hipSuccess) return err;
  const size_t nn = size_t(n);
  *total = 4 * align256(8 * nn) + 5 * align256(4 * nn) + 2 * align256(4 * (nn + 1)) +
           align256(std::max(sb, cb));
  *sort_bytes = sb;
  *scan_bytes = cb;
  return hipSuccess;
}

static VoxScratch carve(void *base, int64_t n, size_t temp_bytes) {
  char *p = static_cast<char *>(base);
  const size_t nn = size_t(n);
  VoxScratch s;
  s.keys_in = reinterpret_cast<uint64_t *>(p);
  p += align256(8 * nn);
  s.keys_out = reinterpret_cast<uint64_t *>(p);
  p += align256(8 * nn);
  s.bsort_in = reinterpret_cast<uint64_t *>(p);
  p += align256(8 * nn);
  s.bsort_out = reinterpret_cast<uint64_t *>(p);
  p += align256(8 * nn);
  s.idx_in = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.idx_out = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.head = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.ord1 = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.spare = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.seg = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * (nn + 1));
  s.bstart = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * (nn + 1));
  s.temp = p;
  s.temp_bytes = temp_bytes;
  return s;
}

// Host driver used by vgicp_voxelize.  Returns a status code and fills *map.
int voxelize_impl(vgicp_ctx ctx, const vgicp_cloud *cloud, double resolution, vgicp_map *out,
                  std::string &msg);

}  // namespace vgicp

// ---------------------------------------------------------------------------

#define HIP_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) {                                                   \
      msg = std::string(#expr) + ": " + hipGetErrorString(_e);                \
      return _e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP;           \
    }                                                                         \
  } while (0)

namespace vgicp {

static int ensure_scratch(vgicp_ctx ctx, size_t bytes, std::string &msg) {
  if (ctx->scratch_bytes >= bytes) return VGICP_OK;
  if (ctx->scratch) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipFree(ctx->scratch));
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  const size_t want = std::max(bytes, size_t(1) << 20);
  HIP_TRY(hipMalloc(&ctx->scratch, want));
  ctx->scratch_bytes = want;
  return VGICP_OK;
}

int voxelize_impl(vgicp_ctx ctx, const vgicp_cloud *cloud, double resolution, vgicp_map *out,
                  std::string &msg) {
  const int64_t n = cloud->n;
  const float s = float(1.0 / resolution);
  const hipStream_t st = ctx->stream;

  int64_t n_voxels = 0;
  VoxScratch sc{};
  if (n > 0) {
    size_t total = 0, sort_bytes = 0, scan_bytes = 0;
    HIP_TRY(plan_scratch(n, st, &total, &sort_bytes, &scan_bytes));
    int rc = ensure_scratch(ctx, total, msg);
    if (rc != VGICP_OK) return rc;
    sc = carve(ctx->scratch, n, std::max(sort_bytes, scan_bytes));

    HIP_TRY(hipMemsetAsync(ctx->err_word, 0, sizeof(uint32_t), st));
    k_voxel_keys<<<grid_for(n), 256, 0, st>>>(cloud->xyz, n, s, sc.keys_in, sc.idx_in,
                                               ctx->err_word);
    HIP_TRY(hipGetLastError());
    size_t tb = sc.temp_bytes;
    HIP_TRY(rocprim::radix_sort_pairs(sc.temp, tb, sc.keys_in, sc.keys_out, sc.idx_in, sc.idx_out,
                                      size_t(n), 0, 63, st));
    k_segment_heads<<<grid_for(n), 256, 0, st>>>(sc.keys_out, n, sc.head);
    HIP_TRY(hipGetLastError());
    tb = sc.temp_bytes;
    HIP_TRY(rocprim::inclusive_scan(sc.temp, tb, sc.head, sc.ord1, size_t(n),
                                    rocprim::plus<uint32_t>(), st));
    k_segment_starts<<<grid_for(n), 256, 0, st>>>(sc.head, sc.ord1, n, sc.seg);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ctx->host_pinned, ctx->err_word, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(ctx->host_pinned + 1, sc.ord1 + (n - 1), sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const uint32_t err = ctx->host_pinned[0];
    if (err & kErrNonFinite) {
      msg = "vgicp_voxelize: a point coordinate is not finite";
      return VGICP_ENONFINITE;
    }
    if (err & kErrRange) {
      msg = "vgicp_voxelize: a voxel key lies outside [-2^20, 2^20)";
      return VGICP_ERANGE;
    }
    n_voxels = int64_t(ctx->host_pinned[1]);
  }

  // Brick order: sort the voxels by (brick key, position in the brick).
  int64_t n_bricks = 0;
  uint64_t *vkey = sc.keys_in;
  uint32_t *vord_in = sc.idx_in, *bhead = sc.head, *bord1 = sc.ord1, *vord_out = sc.spare;
  if (n_voxels > 0) {
    size_t need_sort = 0, need_scan = 0;
    HIP_TRY(rocprim::radix_sort_pairs(nullptr, need_sort, (uint64_t *)nullptr,
                                      (uint64_t *)nullptr, (uint32_t *)nullptr,
                                      (uint32_t *)nullptr, size_t(n_voxels), 0, 63, st));
    HIP_TRY(rocprim::inclusive_scan(nullptr, need_scan, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                    size_t(n_voxels), rocprim::plus<uint32_t>(), st));
    // rocPRIM's temporary storage for V <= n elements normally fits in the
    // storage planned for n; if it does not, this phase gets its own.
    void *temp = sc.temp;
    size_t temp_bytes = sc.temp_bytes;
    void *own_temp = nullptr;
    if (need_sort > temp_bytes || need_scan > temp_bytes) {
      temp_bytes = std::max(need_sort, need_scan);
      HIP_TRY(hipMalloc(&own_temp, temp_bytes));
      temp = own_temp;
    }
    const int64_t V = n_voxels;
    k_brick_sortkeys<<<grid_for(V), 256, 0, st>>>(sc.keys_out, sc.seg, V, vkey, sc.bsort_in,
                                                   vord_in);
    HIP_TRY(hipGetLastError());
    size_t tb = temp_bytes;
    hipError_t pe = rocprim::radix_sort_pairs(temp, tb, sc.bsort_in, sc.bsort_out, vord_in,
                                              vord_out, size_t(V), 0, 63, st);
    if (pe == hipSuccess) {
      k_brick_heads<<<grid_for(V), 256, 0, st>>>(sc.bsort_out, V, bhead);
      pe = hipGetLastError();
    }
    tb = temp_bytes;
    if (pe == hipSuccess)
      pe = rocprim::inclusive_scan(temp, tb, bhead, bord1, size_t(V), rocprim::plus<uint32_t>(),
                                   st);
    if (pe == hipSuccess) {
      k_segment_starts<<<grid_for(V), 256, 0, st>>>(bhead, bord1, V, sc.bstart);
      pe = hipGetLastError();
    }
    if (pe == hipSuccess)
      pe = hipMemcpyAsync(ctx->host_pinned + 1, bord1 + (V - 1), sizeof(uint32_t),
                          hipMemcpyDeviceToHost, st);
    if (pe == hipSuccess) pe = hipStreamSynchronize(st);
    if (own_temp) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(own_temp);
    }
    HIP_TRY(pe);
    n_bricks = int64_t(ctx->host_pinned[1]);
  }

  // Load factor at most 1/8: a lookup in an empty brick (most misses of a
  // partial overlap) almost always stops at an empty home record or one
  // probe later.  At most kMaxMapBricks bricks, so the table (at most 2^27
  // records) stays within 32-bit byte offsets.
  if (n_bricks > kMaxMapBricks) {
    msg = "vgicp_voxelize: more than 2^24 occupied bricks in one map";
    return VGICP_EINVAL;
  }
  int64_t cap = 16;
  uint32_t log2cap = 4;
  while (cap < 8 * n_bricks) {
    cap <<= 1;
    ++log2cap;
  }
  vgicp_map m = new (std::nothrow) vgicp_voxelmap_s();
  if (!m) {
    msg = "vgicp_voxelize: out of host memory";
    return VGICP_ENOMEM;
  }
  m->device = ctx->device;
  m->n_voxels = n_voxels;
  m->n_bricks = n_bricks;
  m->capacity = cap;
  m->log2cap = log2cap;
  m->scale = s;
  m->resolution = resolution;
  const size_t brick_bytes = align256(size_t(cap) * sizeof(BrickRecord));
  const uint32_t obits = occ_bits(cap);
  const size_t occ_bytes = align256(size_t(obits / 8));
  const size_t stats_bytes = align256(size_t(n_voxels) * sizeof(VoxelStats));
  hipError_t e = hipMalloc(&m->buffer, brick_bytes + occ_bytes + stats_bytes +
                                           size_t(n_voxels) * sizeof(VoxelInfo));
  if (e == hipSuccess) {
    char *base = static_cast<char *>(m->buffer);
    m->bricks = reinterpret_cast<BrickRecord *>(base);
    m->occ = reinterpret_cast<uint32_t *>(base + brick_bytes);
    m->stats = reinterpret_cast<VoxelStats *>(base + brick_bytes + occ_bytes);
    m->info = reinterpret_cast<VoxelInfo *>(base + brick_bytes + occ_bytes + stats_bytes);
  }
  if (e != hipSuccess) {
    delete m;
    msg = std::string("vgicp_voxelize: hipMalloc of the voxel map: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP;
  }
  k_fill_empty<<<grid_for(std::max<int64_t>(cap, obits / 32)), 256, 0, st>>>(
      m->bricks, cap, m->occ, obits / 32);
  if (n_voxels > 0) {
    k_build_bricks<<<grid_for(n_bricks), 256, 0, st>>>(sc.bsort_out, sc.bstart, n_bricks,
                                                       n_voxels, m->bricks, log2cap, m->occ,
                                                       obits - 1);
    k_build_payload<<<grid_for(n_voxels), 256, 0, st>>>(cloud->xyz, cloud->cov, n, sc.idx_out,
                                                        sc.seg, vord_out, vkey, n_voxels,
                                                        m->stats, m->info);
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipFree(m->buffer);
    delete m;
    msg = std::string("vgicp_voxelize: kernel launch: ") + hipGetErrorString(e);
    return VGICP_EHIP;
  }
  *out = m;
  return VGICP_OK;
}

int map_export_impl(vgicp_ctx ctx, vgicp_map m, int32_t *keys, float *mean, float *cov,
                    int32_t *count, std::string &msg) {
  if (m->n_voxels == 0) return VGICP_OK;
  k_export<<<grid_for(m->n_voxels), 256, 0, ctx->stream>>>(m->stats, m->info, m->n_voxels, keys,
                                                           mean,
                                                           cov, count);
  HIP_TRY(hipGetLastError());
  return VGICP_OK;
}

}  // namespace vgicp
