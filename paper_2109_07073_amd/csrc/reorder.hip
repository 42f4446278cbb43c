// Resident, spatially ordered copies of the source clouds of a factor set.
//
// A linearization round streams every source point once and gathers the
// target voxel of each (Sec. III-A).  Consecutive points of a scan in its
// recorded order can lie far apart (a ring of a rotating sensor, thinned),
// so the 64 lanes of a wave touch many brick records and voxel statistics
// lines.  A factor set therefore keeps its own copy of each source cloud with
// the points in Morton order of cells at the finest resolution among the maps
// the cloud is matched against: neighbours in memory are neighbours in space,
// and a rigid transform keeps them neighbours in the target map.  The copy is
// made once; every round reads it instead of the caller's arrays.  Per-point
// outputs are written at the caller's index through the stored permutation.
// The results are the same up to FP32 summation order (integer outputs are
// identical).

#include "vgicp_internal.hpp"

#include <rocprim/device/device_radix_sort.hpp>

namespace vgicp {
namespace {

constexpr int kThreads = 256;
constexpr float kCellLo = -1048576.0f;  // -2^20
constexpr float kCellHi = 1048575.0f;   //  2^20 - 1

// Cell index on one axis, offset to [0, 2^21); NaN and out-of-range values
// clamp to the ends (any order of such points is valid).
__device__ __forceinline__ uint32_t cell21(float x, float inv_cell) {
  const float q = fminf(fmaxf(floorf(x * inv_cell), kCellLo), kCellHi);
  return uint32_t(int32_t(q) + 1048576);
}

// The 21 low bits of v moved to every third bit (bit k to bit 3k).
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// Morton key (63 bits, x most significant within each bit triple) and the
// point's own index of every point of one cloud.
__global__ void __launch_bounds__(kThreads)
k_morton_keys(const float *__restrict__ xyz, uint32_t n, float inv_cell,
              uint64_t *__restrict__ keys, uint32_t *__restrict__ idx) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const uint32_t cx = cell21(xyz[i], inv_cell);
  const uint32_t cy = cell21(xyz[uint64_t(n) + i], inv_cell);
  const uint32_t cz = cell21(xyz[2ull * n + i], inv_cell);
  keys[i] = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
  idx[i] = i;
}

// Copy point perm[i] of the cloud to position i of the ordered copy
// (three coordinates and six covariance entries per point), and
// count the points with a non-finite coordinate (nonfinite[0]) or covariance
// entry (nonfinite[1]): the only full pass over a factor set's inputs.
__global__ void __launch_bounds__(kThreads)
k_gather_points(const float *__restrict__ xyz, const float *__restrict__ cov, uint32_t n,
                const int32_t *__restrict__ perm, float *__restrict__ xyz_out,
                float *__restrict__ cov_out, unsigned long long *__restrict__ nonfinite) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const uint64_t j = uint32_t(perm[i]);
  const float x = xyz[j], y = xyz[uint64_t(n) + j], z = xyz[2ull * n + j];
  xyz_out[3ull * i] = x;
  xyz_out[3ull * i + 1] = y;
  xyz_out[3ull * i + 2] = z;
  const float2 *src = reinterpret_cast<const float2 *>(cov + 6 * j);
  float2 *dst = reinterpret_cast<float2 *>(cov_out + 6ull * i);
  const float2 c0 = src[0], c1 = src[1], c2 = src[2];
  dst[0] = c0;
  dst[1] = c1;
  dst[2] = c2;
  const bool bad_p = !(isfinite(x) && isfinite(y) && isfinite(z));
  const bool bad_c = !(isfinite(c0.x) && isfinite(c0.y) && isfinite(c1.x) && isfinite(c1.y) &&
                       isfinite(c2.x) && isfinite(c2.y));
  if (bad_p) atomicAdd(&nonfinite[0], 1ull);
  if (bad_c) atomicAdd(&nonfinite[1], 1ull);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Position q of the sorted (factor, voxel) keys is point q - corr_offset of
// factor f = key >> 32 in its new copy; it takes point vals[q] of the old
// copy (coordinates, covariance, and the caller's index through the old
// permutation, or vals[q] itself when the old copy is the caller's cloud).
__global__ void __launch_bounds__(kThreads)
k_gather_factor_points(const FactorDesc *__restrict__ old_desc,
                       const FactorDesc *__restrict__ new_desc, const uint64_t *__restrict__ keys,
                       const uint32_t *__restrict__ vals, uint64_t total) {
  const uint64_t q = uint64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= total) return;
  const uint32_t f = uint32_t(keys[q] >> 32);
  const uint64_t i = vals[q];
  const FactorDesc &o = old_desc[f];
  const FactorDesc &d = new_desc[f];
  const uint64_t local = q - uint64_t(d.corr_offset);
  float *xyz = const_cast<float *>(d.xyz);
  xyz[3 * local] = o.xyz[3 * i];
  xyz[3 * local + 1] = o.xyz[3 * i + 1];
  xyz[3 * local + 2] = o.xyz[3 * i + 2];
  const float2 *src = reinterpret_cast<const float2 *>(o.cov + 6 * i);
  float2 *dst = reinterpret_cast<float2 *>(const_cast<float *>(d.cov) + 6 * local);
  dst[0] = src[0];
  dst[1] = src[1];
  dst[2] = src[2];
  const_cast<int32_t *>(d.perm)[local] = o.perm ? o.perm[i] : int32_t(i);
}

// Coordinates of a caller's cloud ([3][n], one plane per axis) point by point
// ([n][3]), the layout the lookup kernels read.
__global__ void __launch_bounds__(kThreads)
k_interleave_xyz(const float *__restrict__ planes, uint32_t n, float *__restrict__ out) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  out[3ull * i] = planes[i];
  out[3ull * i + 1] = planes[uint64_t(n) + i];
  out[3ull * i + 2] = planes[2ull * n + i];
}

}  // namespace

hipError_t launch_interleave_xyz(const float *planes, int64_t n, float *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const uint32_t grid = uint32_t((uint64_t(n) + kThreads - 1) / kThreads);
  k_interleave_xyz<<<grid, kThreads, 0, st>>>(planes, uint32_t(n), out);
  return hipGetLastError();
}

hipError_t launch_voxel_order_keys(const vgicp_factorset_s *fs, const double *poses,
                                   uint64_t *keys, uint32_t *vals, hipStream_t st);

hipError_t reorder_by_target(vgicp_factorset_s *fs, const double *poses, hipStream_t st) {
  const int64_t total = fs->total_points;
  if (fs->n_factors == 0 || total == 0) return hipSuccess;
  // new per-factor copies: covariances [n][6], coordinates [n][3], permutation [n]
  std::vector<FactorDesc> nd = fs->h_factors;
  size_t bytes = 0;
  std::vector<size_t> off(nd.size(), 0);
  for (size_t f = 0; f < nd.size(); ++f) {
    const size_t n = size_t(nd[f].n);
    off[f] = bytes;
    if (n) bytes += align256(24 * n) + align256(12 * n) + align256(4 * n);
  }
  int end_bit = 32;
  while (end_bit < 64 && (uint64_t(fs->n_factors - 1) >> (end_bit - 32)) != 0) ++end_bit;
  size_t sort_bytes = 0;
  hipError_t e = rocprim::radix_sort_pairs(
      nullptr, sort_bytes, static_cast<const uint64_t *>(nullptr), static_cast<uint64_t *>(nullptr),
      static_cast<const uint32_t *>(nullptr), static_cast<uint32_t *>(nullptr), size_t(total), 0,
      end_bit, st);
  if (e != hipSuccess) return e;
  const size_t kb = align256(8 * size_t(total)), vb = align256(4 * size_t(total));
  const size_t db = align256(sizeof(FactorDesc) * nd.size());
  char *buf = nullptr, *tmp = nullptr;
  e = hipMalloc(&buf, std::max<size_t>(bytes, 1));
  if (e == hipSuccess) e = hipMalloc(&tmp, 2 * kb + 2 * vb + db + align256(sort_bytes));
  if (e != hipSuccess) {
    if (buf) (void)hipFree(buf);
    return e;
  }
  for (size_t f = 0; f < nd.size(); ++f) {
    const size_t n = size_t(nd[f].n);
    char *p = buf + off[f];
    nd[f].cov = n ? reinterpret_cast<float *>(p) : nullptr;
    nd[f].xyz = n ? reinterpret_cast<float *>(p + align256(24 * n)) : nullptr;
    nd[f].perm = n ? reinterpret_cast<int32_t *>(p + align256(24 * n) + align256(12 * n)) : nullptr;
  }
  uint64_t *keys_in = reinterpret_cast<uint64_t *>(tmp);
  uint64_t *keys_out = reinterpret_cast<uint64_t *>(tmp + kb);
  uint32_t *vals_in = reinterpret_cast<uint32_t *>(tmp + 2 * kb);
  uint32_t *vals_out = reinterpret_cast<uint32_t *>(tmp + 2 * kb + vb);
  FactorDesc *d_new = reinterpret_cast<FactorDesc *>(tmp + 2 * kb + 2 * vb);
  void *sort_tmp = tmp + 2 * kb + 2 * vb + db;
  e = launch_voxel_order_keys(fs, poses, keys_in, vals_in, st);
  if (e == hipSuccess)
    e = rocprim::radix_sort_pairs(sort_tmp, sort_bytes, keys_in, keys_out, vals_in, vals_out,
                                  size_t(total), 0, end_bit, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_new, nd.data(), sizeof(FactorDesc) * nd.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    const uint64_t grid = (uint64_t(total) + kThreads - 1) / kThreads;
    k_gather_factor_points<<<unsigned(grid), kThreads, 0, st>>>(fs->d_factors, d_new, keys_out,
                                                                vals_out, uint64_t(total));
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(fs->d_factors, nd.data(), sizeof(FactorDesc) * nd.size(),
                       hipMemcpyHostToDevice, st);
  const hipError_t se = hipStreamSynchronize(st);
  if (e == hipSuccess) e = se;
  (void)hipFree(tmp);
  if (e != hipSuccess) {
    // the device descriptors may already name the new copies: put the old ones back
    (void)hipMemcpy(fs->d_factors, fs->h_factors.data(), sizeof(FactorDesc) * nd.size(),
                    hipMemcpyHostToDevice);
    (void)hipFree(buf);
    return e;
  }
  if (fs->d_sorted) (void)hipFree(fs->d_sorted);
  fs->d_sorted = buf;
  fs->h_factors = nd;
  return hipSuccess;
}

hipError_t make_sorted_sources(const vgicp_cloud *sources, int32_t n_sources,
                               const std::vector<double> &cell, void **buffer,
                               std::vector<SortedSource> &out, hipStream_t st,
                               int64_t *nonfinite) {
  *buffer = nullptr;
  if (nonfinite) nonfinite[0] = nonfinite[1] = 0;
  out.assign(size_t(n_sources), SortedSource{});
  // layout: per used cloud, covariances [n][6], coordinates [n][3], permutation [n]
  size_t total = 0;
  uint32_t nmax = 0;
  std::vector<size_t> off(size_t(n_sources), 0);
  for (int32_t s = 0; s < n_sources; ++s) {
    const int64_t n = sources[s].n;
    if (!(cell[size_t(s)] > 0.0) || n <= 0) continue;
    off[size_t(s)] = total;
    total += align256(24 * size_t(n)) + align256(12 * size_t(n)) + align256(4 * size_t(n));
    nmax = std::max(nmax, uint32_t(n));
  }
  if (total == 0) return hipSuccess;

  size_t sort_bytes = 0;
  for (int32_t s = 0; s < n_sources; ++s) {
    if (!(cell[size_t(s)] > 0.0) || sources[s].n <= 0) continue;
    size_t b = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, b, static_cast<const uint64_t *>(nullptr),
                                             static_cast<uint64_t *>(nullptr),
                                             static_cast<const uint32_t *>(nullptr),
                                             static_cast<uint32_t *>(nullptr),
                                             uint32_t(sources[s].n), 0, 63, st);
    if (e != hipSuccess) return e;
    sort_bytes = std::max(sort_bytes, b);
  }
  const size_t kbytes = align256(8 * size_t(nmax));
  const size_t ibytes = align256(4 * size_t(nmax));
  char *tmp = nullptr;
  hipError_t e = hipMalloc(buffer, total);
  if (e == hipSuccess) e = hipMalloc(&tmp, 2 * kbytes + ibytes + align256(sort_bytes) + 256);
  if (e != hipSuccess) {
    if (*buffer) (void)hipFree(*buffer);
    *buffer = nullptr;
    return e;
  }
  uint64_t *keys_in = reinterpret_cast<uint64_t *>(tmp);
  uint64_t *keys_out = reinterpret_cast<uint64_t *>(tmp + kbytes);
  uint32_t *idx_in = reinterpret_cast<uint32_t *>(tmp + 2 * kbytes);
  void *sort_tmp = tmp + 2 * kbytes + ibytes;
  unsigned long long *d_bad =
      reinterpret_cast<unsigned long long *>(tmp + 2 * kbytes + ibytes + align256(sort_bytes));
  e = hipMemsetAsync(d_bad, 0, 2 * sizeof(unsigned long long), st);

  char *base = static_cast<char *>(*buffer);
  for (int32_t s = 0; s < n_sources && e == hipSuccess; ++s) {
    const vgicp_cloud &c = sources[s];
    if (!(cell[size_t(s)] > 0.0) || c.n <= 0) continue;
    const uint32_t n = uint32_t(c.n);
    char *p = base + off[size_t(s)];
    float *cov_s = reinterpret_cast<float *>(p);
    float *xyz_s = reinterpret_cast<float *>(p + align256(24 * size_t(n)));
    int32_t *perm = reinterpret_cast<int32_t *>(p + align256(24 * size_t(n)) + align256(12 * size_t(n)));
    const uint32_t grid = (n + kThreads - 1) / kThreads;
    k_morton_keys<<<grid, kThreads, 0, st>>>(c.xyz, n, float(1.0 / cell[size_t(s)]), keys_in, idx_in);
    e = hipGetLastError();
    size_t b = align256(sort_bytes);
    if (e == hipSuccess)
      e = rocprim::radix_sort_pairs(sort_tmp, b, keys_in, keys_out, idx_in,
                                    reinterpret_cast<uint32_t *>(perm), n, 0, 63, st);
    if (e == hipSuccess) {
      k_gather_points<<<grid, kThreads, 0, st>>>(c.xyz, c.cov, n, perm, xyz_s, cov_s, d_bad);
      e = hipGetLastError();
    }
    out[size_t(s)] = SortedSource{xyz_s, cov_s, perm};
  }
  // the temporaries are reused cloud after cloud on the stream; free them
  // once the last gather has run
  unsigned long long bad[2] = {0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, st);
  const hipError_t se = hipStreamSynchronize(st);
  if (e == hipSuccess) e = se;
  if (e == hipSuccess && nonfinite) {
    nonfinite[0] = int64_t(bad[0]);
    nonfinite[1] = int64_t(bad[1]);
  }
  (void)hipFree(tmp);
  if (e != hipSuccess) {
    (void)hipFree(*buffer);
    *buffer = nullptr;
    out.assign(size_t(n_sources), SortedSource{});
  }
  return e;
}

}  // namespace vgicp
