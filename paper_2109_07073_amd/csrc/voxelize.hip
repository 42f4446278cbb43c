// Voxel-map construction on gfx950 (Sec. III-A, VGICP voxel data association).
//
// A cloud becomes an open-addressed hash table keyed by the packed voxel key
// (a key array and a payload array indexed by slot).  Each payload carries
// the voxel mean and the mean of the point covariances (the VGICP aggregation
// of point distributions), both accumulated in FP64 in point order and
// rounded once to FP32.
//
// Steps: keys -> radix sort of (key, point index) -> segment heads -> scan
// -> segment starts -> [one host sync to size the table] -> FP64 segment sums
// and hash insertion.  This runs once per cloud, off the per-iteration path.

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

__global__ void __launch_bounds__(256) k_fill_empty(uint64_t *__restrict__ keys, int64_t cap) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < cap) keys[i] = kEmptyKey;
}

// One thread per voxel: sequential FP64 sums over the voxel's points in point
// order, one FP64 division, one rounding to FP32, then linear-probing insert.
__global__ void __launch_bounds__(256)
k_build_slots(const float *__restrict__ xyz, const float *__restrict__ cov, int64_t n,
              const uint64_t *__restrict__ sorted_keys, const uint32_t *__restrict__ sorted_idx,
              const uint32_t *__restrict__ seg, int64_t n_voxels, uint64_t *__restrict__ keys,
              Payload *__restrict__ payload, uint32_t log2cap) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n_voxels) return;
  const uint32_t b = seg[v], e = seg[v + 1];
  double sm[3] = {0.0, 0.0, 0.0};
  double sc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (uint32_t j = b; j < e; ++j) {
    const uint32_t p = sorted_idx[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) sm[a] += double(xyz[a * n + p]);
#pragma unroll
    for (int a = 0; a < 6; ++a) sc[a] += double(cov[a * n + p]);
  }
  const double cnt = double(e - b);
  const uint64_t key = sorted_keys[b];
  const uint32_t mask = (1u << log2cap) - 1u;
  uint32_t h = hash_slot(key, log2cap);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev =
        atomicCAS(reinterpret_cast<unsigned long long *>(&keys[h]),
                  (unsigned long long)kEmptyKey, (unsigned long long)key);
    if (prev == kEmptyKey) break;
    h = (h + 1u) & mask;
  }
  Payload pl;
#pragma unroll
  for (int a = 0; a < 3; ++a) pl.mean[a] = float(sm[a] / cnt);
#pragma unroll
  for (int a = 0; a < 6; ++a) pl.cov[a] = float(sc[a] / cnt);
  pl.ordinal = int32_t(v);
  pl.count = int32_t(e - b);
#pragma unroll
  for (int a = 0; a < 5; ++a) pl.pad[a] = 0;
  payload[h] = pl;
}

__global__ void __launch_bounds__(256)
k_export(const uint64_t *__restrict__ keys_tab, const Payload *__restrict__ payload, int64_t cap,
         int32_t *__restrict__ keys, float *__restrict__ mean, float *__restrict__ cov,
         int32_t *__restrict__ count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  const uint64_t key = keys_tab[i];
  if (key == kEmptyKey) return;
  const Payload s = payload[i];
  const int64_t o = s.ordinal;
  if (keys) {
#pragma unroll
    for (int a = 0; a < 3; ++a) keys[3 * o + a] = key_field(key, a);
  }
  if (mean) {
#pragma unroll
    for (int a = 0; a < 3; ++a) mean[3 * o + a] = s.mean[a];
  }
  if (cov) {
#pragma unroll
    for (int a = 0; a < 6; ++a) cov[6 * o + a] = s.cov[a];
  }
  if (count) count[o] = s.count;
}

static inline unsigned grid_for(int64_t n, int block = 256) {
  return unsigned((n + block - 1) / block);
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch layout for n points; returns total bytes (rocPRIM temp included).
struct VoxScratch {
  uint64_t *keys_in, *keys_out;
  uint32_t *idx_in, *idx_out, *head, *ord1, *seg;
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
  *total = 2 * align256(8 * nn) + 5 * align256(4 * nn) + align256(4 * (nn + 1)) +
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
  s.idx_in = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.idx_out = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.head = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  s.ord1 = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * nn);
  p += align256(4 * nn);  // spare
  s.seg = reinterpret_cast<uint32_t *>(p);
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

  // Load factor at most 1/8: a lookup that misses (most points of a partial
  // overlap) then almost always finds an empty home slot or one more probe.
  // Slots are int32 indices, so the table stops at 2^31 slots (load <= 1/2).
  int64_t cap = 16;
  uint32_t log2cap = 4;
  while (cap < 8 * n_voxels && cap < (int64_t(1) << 31)) {
    cap <<= 1;
    ++log2cap;
  }
  if (cap < 2 * n_voxels) {
    msg = "vgicp_voxelize: more than 2^30 voxels in one map";
    return VGICP_EINVAL;
  }
  vgicp_map m = new (std::nothrow) vgicp_voxelmap_s();
  if (!m) {
    msg = "vgicp_voxelize: out of host memory";
    return VGICP_ENOMEM;
  }
  m->device = ctx->device;
  m->n_voxels = n_voxels;
  m->capacity = cap;
  m->log2cap = log2cap;
  m->scale = s;
  m->resolution = resolution;
  const size_t key_bytes = (size_t(cap) * sizeof(uint64_t) + 255) & ~size_t(255);
  hipError_t e = hipMalloc(&m->buffer, key_bytes + size_t(cap) * sizeof(Payload));
  if (e == hipSuccess) {
    m->keys = static_cast<uint64_t *>(m->buffer);
    m->payload = reinterpret_cast<Payload *>(static_cast<char *>(m->buffer) + key_bytes);
  }
  if (e != hipSuccess) {
    delete m;
    msg = std::string("vgicp_voxelize: hipMalloc of the hash table: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VGICP_ENOMEM : VGICP_EHIP;
  }
  k_fill_empty<<<grid_for(cap), 256, 0, st>>>(m->keys, cap);
  if (n_voxels > 0) {
    k_build_slots<<<grid_for(n_voxels), 256, 0, st>>>(cloud->xyz, cloud->cov, n, sc.keys_out,
                                                       sc.idx_out, sc.seg, n_voxels, m->keys,
                                                       m->payload, log2cap);
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
  k_export<<<grid_for(m->capacity), 256, 0, ctx->stream>>>(m->keys, m->payload, m->capacity, keys,
                                                           mean, cov, count);
  HIP_TRY(hipGetLastError());
  return VGICP_OK;
}

}  // namespace vgicp
