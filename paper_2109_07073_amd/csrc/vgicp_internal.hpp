// Internal definitions shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vgicp.h"

namespace vgicp {

// ---------------------------------------------------------------- voxel keys
// Keys are packed as three biased 21-bit fields (kx, ky, kz) in the low 63
// bits, kx highest, so numeric order of packed keys is lexicographic key
// order.  All-ones marks an empty hash slot (bit 63 is never set by a key).
constexpr int kKeyBits = 21;
constexpr int32_t kKeyLimit = 1 << 20;  // keys lie in [-2^20, 2^20)
constexpr float kKeyLimitF = 1048576.0f;
constexpr uint64_t kEmptyKey = ~0ull;

__host__ __device__ inline uint64_t pack_key(int32_t kx, int32_t ky, int32_t kz) {
  return (uint64_t(uint32_t(kx + kKeyLimit)) << (2 * kKeyBits)) |
         (uint64_t(uint32_t(ky + kKeyLimit)) << kKeyBits) | uint64_t(uint32_t(kz + kKeyLimit));
}

__host__ __device__ inline int32_t key_field(uint64_t key, int which) {
  const int shift = (2 - which) * kKeyBits;
  return int32_t((key >> shift) & ((1u << kKeyBits) - 1)) - kKeyLimit;
}

// ---------------------------------------------------------------- bricks
// Voxels are grouped in bricks of 4 x 4 x 4.  A voxel's bit in its brick's
// 64-bit occupancy mask interleaves the low two bits of its key per axis
// (x1 y1 z1 x0 y0 z0, Morton order), so the voxels of a 2 x 2 x 2 corner of
// a brick are consecutive in the dense per-voxel arrays.  Consecutive points
// of a scan mostly fall in the same or neighbouring bricks, so their lookups
// share brick records (and cache lines) instead of scattering over a
// voxel-keyed table.
//
// A brick is named by one field per axis, floor(k / 4) + 2^18 + 1, which is
// in [1, 2^19] for keys in [-2^20, 2^20).  A lookup clamps the scaled
// coordinate to [-2^20 - 4, 2^20] instead of testing the range, so a point
// outside the key range (or NaN) gets field 0 or 2^19 + 1: a brick no map
// holds.  Record keys pack the fields in 20 bits each (60 bits, never
// kEmptyKey).
constexpr int kBrickBits = 20;
constexpr int32_t kBrickBias = (1 << 18) + 1;
constexpr float kClampLoF = -1048580.0f;  // -2^20 - 4
constexpr float kClampHiF = 1048576.0f;   // 2^20

__host__ __device__ inline uint32_t brick_field(int32_t k) {
  return uint32_t((k >> 2) + kBrickBias);
}

__host__ __device__ inline uint64_t brick_key(uint32_t fx, uint32_t fy, uint32_t fz) {
  return (uint64_t(fx) << (2 * kBrickBits)) | (uint64_t(fy) << kBrickBits) | uint64_t(fz);
}

// Bits of b taken where m is set, the others from a (one v_bfi_b32).
__host__ __device__ inline uint32_t bit_select(uint32_t m, uint32_t b, uint32_t a) {
  return (b & m) | (a & ~m);
}

// The two low bits of each key spread three apart by a multiply: (k & 3) * 5
// holds bit 0 at bits 0 and 2 and bit 1 at bits 1 and 3, so (k & 3) * 20 has
// x0, x1 at bits 2, 5 (mask 0x24), (k & 3) * 10 has y0, y1 at bits 1, 4 (mask
// 0x12) and (k & 3) * 5 has z0, z1 at bits 0, 3 (mask 0x09).
__host__ __device__ inline uint32_t brick_bit(int32_t kx, int32_t ky, int32_t kz) {
  const uint32_t x = uint32_t(kx & 3) * 20u, y = uint32_t(ky & 3) * 10u, z = uint32_t(kz & 3) * 5u;
  return bit_select(0x24u, x, bit_select(0x12u, y, z & 0x0fu));
}

// Brick-major sort key of an in-range voxel: the brick fields less one (19
// bits each, 57 bits) above the voxel's bit in the brick.
__host__ __device__ inline uint64_t brick_sort_key(int32_t kx, int32_t ky, int32_t kz) {
  const uint64_t g = (uint64_t(brick_field(kx) - 1u) << 38) |
                     (uint64_t(brick_field(ky) - 1u) << 19) | uint64_t(brick_field(kz) - 1u);
  return (g << 6) | uint64_t(brick_bit(kx, ky, kz));
}

__host__ __device__ inline uint64_t brick_key_of_sort_key(uint64_t sk) {
  const uint64_t g = sk >> 6;
  const uint32_t m = (1u << 19) - 1u;
  return brick_key(uint32_t(g >> 38) + 1u, (uint32_t(g >> 19) & m) + 1u, (uint32_t(g) & m) + 1u);
}

// Home record of a brick.  The four bricks of a 2 x 2 x 1 group (fields x
// and y halved) share one 128-byte line of four records, each at the position
// given by the low bits of its x and y fields, so the bricks a wave's points
// touch fall in few lines.  The line is a linear combination of the group's
// coordinates with odd 24-bit multipliers (full-rate 24-bit multiplies on
// gfx950) folded to 32 bits, spread by a 32-bit Fibonacci multiply.  Probing
// steps one line on, at the same position.  Replaying 40 scan factors on the
// CPU, a 64-point wave touches 6.0 record lines here against 9.7 for one
// record per hashed brick, and about 1 % of waves probe past a home record.
constexpr uint32_t kProbeStep = 4;

__host__ __device__ inline uint32_t brick_slot(uint32_t fx, uint32_t fy, uint32_t fz,
                                               uint32_t log2cap) {
  const uint32_t k = fz + ((fy >> 1) & 0xffffffu) * 353u + ((fx >> 1) & 0xffffffu) * 294913u;
  // the line, (k * 0x9E3779B9) >> (34 - log2cap), shifted left by two
  const uint32_t line4 = (k * 0x9E3779B9u) >> (32 - log2cap);
  return bit_select(~3u, line4, bit_select(2u, fy << 1, fx));
}

__host__ __device__ inline uint32_t brick_slot_of_key(uint64_t bkey, uint32_t log2cap) {
  const uint32_t m = (1u << kBrickBits) - 1u;
  return brick_slot(uint32_t(bkey >> (2 * kBrickBits)) & m, uint32_t(bkey >> kBrickBits) & m,
                    uint32_t(bkey) & m, log2cap);
}

// Occupancy bitset of a map's brick table: bit (h mod B) is set when record h
// holds a brick, B = min(cap, kOccMaxBits) (at least 32).  A lookup whose home
// record's bit is clear misses without reading the record (linear probing
// never passes an empty record); a table larger than kOccMaxBits folds its
// slots onto the bits, which only lets some lookups read their record.
constexpr uint32_t kOccMaxBits = 1u << 16;  // 8 KB, staged in LDS per block

__host__ __device__ inline uint32_t occ_bits(int64_t cap) {
  return cap < 32 ? 32u : (cap > int64_t(kOccMaxBits) ? kOccMaxBits : uint32_t(cap));
}

// Size limits that keep every byte offset of a cloud or map within 32 bits
// (the kernels address them through buffer resources).
constexpr int64_t kMaxCloudPoints = int64_t(1) << 26;
constexpr int64_t kMaxMapBricks = int64_t(1) << 24;

// A voxel map is an open-addressed table of brick records (linear probing,
// load factor at most 1/8) plus dense per-voxel arrays:
//   bricks[cap]  32-byte records {brick key (kEmptyKey when free), occupancy
//                mask, index of the brick's first voxel}; a lookup reads key
//                and mask with one 16-byte load and the base with a second
//                load from the same record;
//   stats[V]     what a correspondence reads: mean and covariance, 36 bytes,
//                packed, brick after brick and by mask bit within a brick, so
//                voxel b of a brick sits at base + popcount(mask & (2^b - 1))
//                and the voxels of a scan neighbourhood share cache lines;
//   info[V]      in the same order, what only the map export and the
//                correspondence output read (packed key, ordinal, count).
struct alignas(32) BrickRecord {
  uint64_t key;
  uint64_t mask;
  uint32_t base;
  uint32_t pad[3];
};
static_assert(sizeof(BrickRecord) == 32, "brick record layout");

struct VoxelStats {
  float mean[3];
  float cov[6];  // xx xy xz yy yz zz
};
static_assert(sizeof(VoxelStats) == 36, "voxel statistics layout");

struct alignas(16) VoxelInfo {
  uint64_t key;     // packed voxel key
  int32_t ordinal;  // lexicographic rank of the key
  int32_t count;    // points in the voxel
};
static_assert(sizeof(VoxelInfo) == 16, "voxel info layout");

// ---------------------------------------------------------------- factors
// Tiles.  A 256-thread block of k_linearize looks up kLookupPasses rows of
// 256 points per phase, so tiles that are multiples of kTileQuantum points
// leave no phase partly empty.
constexpr int kLookupPasses = 3;
constexpr int kTileQuantum = 256 * kLookupPasses;
constexpr int kDefaultTile = 6 * kTileQuantum;  // 4608 points

// Bytes of one factor's relative-pose constants in a factor set's table
// (FP32 rotation and translation scaled by 1/r and unscaled, FP64 rotation
// and translation).
constexpr size_t kFactorConstsBytes = 24 * sizeof(float) + 12 * sizeof(double);

// Per-factor device descriptor (read with uniform loads by every tile).
struct FactorDesc {
  const float *xyz;        // [n][3]: a library-owned copy, point by point
  const float *cov;        // [n][6]
  const BrickRecord *bricks;  // target map: brick table
  const VoxelStats *stats;    // target map: per-voxel mean and covariance
  const VoxelInfo *info;      // target map: per-voxel key, ordinal, count
  int64_t n;          // source points (at most kMaxCloudPoints)
  int64_t corr_offset;
  int32_t pose_i;
  int32_t pose_j;
  uint32_t log2cap;
  float scale;        // fl32(1/r) of the target map
  int32_t tile_begin; // first tile of this factor in the tile table
  int32_t n_tiles;    // its tiles: tile_begin + k * tile_stride, k < n_tiles
  uint32_t n_voxels;  // target map: voxels
  const uint32_t *occ;  // target map: occupancy bitset of the brick table
  uint32_t occ_mask;    // occ_bits(cap) - 1
  // Distance between consecutive tiles of this factor in the tile table: 1,
  // or in the interleaved layout the number of factors reading the same
  // source copy.
  int32_t tile_stride;
  // Source points per tile of this factor (its last tile may hold fewer).
  int32_t tile_points;
  // Caller's index of each source point when xyz/cov are a reordered copy of
  // the caller's cloud (per-point outputs are written at it); NULL when the
  // points are in the caller's order.
  const int32_t *perm;
};

// A factor set's ordered copy of one source cloud (Morton order of cells),
// with the caller's index of each point.
struct SortedSource {
  const float *xyz = nullptr;   // [n][3]
  const float *cov = nullptr;   // [n][6]
  const int32_t *perm = nullptr;  // [n]
};

// Coordinates of a caller's cloud, [3][n], copied point by point to out
// ([n][3]) on st.
hipError_t launch_interleave_xyz(const float *planes, int64_t n, float *out, hipStream_t st);

// Ordered copies of the clouds s with cell[s] > 0 and n > 0, in one device
// allocation returned in *buffer (NULL when there is none); out[s] points into
// it.  nonfinite (may be NULL) receives the number of copied points with a
// non-finite coordinate and with a non-finite covariance entry.  Enqueued on
// st and synchronized before returning.
hipError_t make_sorted_sources(const vgicp_cloud *sources, int32_t n_sources,
                               const std::vector<double> &cell, void **buffer,
                               std::vector<SortedSource> &out, hipStream_t st,
                               int64_t *nonfinite = nullptr);

// Replace the source copies of fs by per-factor copies with each factor's
// points in the order of the target voxels they fall in at `poses` (device)
// (points in no voxel last; equal keys keep their order), updating the device
// descriptors.  Synchronizes st.  On failure fs is unchanged.
hipError_t reorder_by_target(vgicp_factorset_s *fs, const double *poses, hipStream_t st);

// One tile: the source points [start, start + tile_points) (at most up to
// the factor's last point) of factor `factor`, whose descriptor holds its
// tile_points.  A padding tile (factor < 0) names no points: the kernels skip
// it and no factor reads its partial sums.
struct Tile {
  int32_t factor;
  int32_t start;
};
constexpr int32_t kPaddingTile = -1;

// Per-tile partial sums written by the linearize/evaluate kernels.
//   [0, 21)  upper triangle (row-major) of the 6x6 source-frame Hessian
//   [21, 27) source-frame gradient
//   27       cost
//   28       inliers
//   29       inliers whose fused covariance was formed in FP64 (linearize and
//            cost kernels)
//   30       inliers whose fused covariance was not positive definite (they
//            add nothing; linearize and cost kernels)
constexpr int kPartialStride = 32;
constexpr int kNumSums = 28;
constexpr int kWideSlot = 29;
constexpr int kDegenerateSlot = 30;
// The pair form's tile partials: 78 upper-triangle entries of the 12 x 12 H
// (row-major), b (12) and the cost, one row of kPairStride doubles per tile;
// its counters use the slots above in the source-frame partials.
constexpr int kNumPairSums = 91;
constexpr int kPairStride = 96;

// Error bits of the device error word.
constexpr uint32_t kErrNonFinite = 1u;
constexpr uint32_t kErrRange = 2u;

// Records `msg` as the last error of ctx (or of the calling thread when ctx
// is NULL) and returns `code`.
int set_error(vgicp_ctx ctx, int code, const std::string &msg);

// Common checks of the calls on a factor set (ctx and fs not NULL, same
// device, poses given when needed); makes ctx's device current.
int check_common(vgicp_ctx ctx, vgicp_factorset fs, const double *poses, const char *who);

// opts (NULL: defaults) validated into *o.
int read_opts(vgicp_ctx ctx, const vgicp_opts *opts, vgicp_opts *o, const char *who);

// Looks up, once per device, the device address of the fixed scratch array
// used by vgicp_linearize_factors_noalloc; `device` must be current.
hipError_t noalloc_setup(int device);

// The poses one batch of a server holds (its max_batch_poses).
int64_t server_max_batch_poses(vgicp_server srv);

}  // namespace vgicp

// Objects behind the opaque handles of the C ABI.
struct vgicp_context_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // Growable scratch for voxelization.
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  uint32_t *err_word = nullptr;       // device
  uint32_t *host_pinned = nullptr;    // pinned host word pair for small readbacks
  int cu_count = 0;
  // Growable workspace of the keyframe calls (vgicp_connect,
  // vgicp_submap_step): device tables and pinned host staging.
  void *map_ws = nullptr;
  size_t map_ws_bytes = 0;
  void *map_host = nullptr;
  size_t map_host_bytes = 0;
  // Kernel timing (see vgicp_ctx_set_timing).
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[VGICP_KERNEL_KINDS];
  double total_ms[VGICP_KERNEL_KINDS] = {0, 0, 0, 0};
  int64_t launches[VGICP_KERNEL_KINDS] = {0, 0, 0, 0};
};

struct vgicp_voxelmap_s {
  int device = 0;
  int64_t n_voxels = 0;
  int64_t capacity = 0;
  uint32_t log2cap = 0;
  float scale = 0.f;
  double resolution = 0.0;
  int64_t n_bricks = 0;
  void *buffer = nullptr;             // one allocation: brick table, stats, info
  vgicp::BrickRecord *bricks = nullptr;
  uint32_t *occ = nullptr;  // occupancy bitset, occ_bits(capacity) bits
  vgicp::VoxelStats *stats = nullptr;
  vgicp::VoxelInfo *info = nullptr;
  int64_t device_bytes() const {
    return capacity * int64_t(sizeof(vgicp::BrickRecord)) + int64_t(vgicp::occ_bits(capacity) / 8) +
           n_voxels * int64_t(sizeof(vgicp::VoxelStats) + sizeof(vgicp::VoxelInfo));
  }
};

struct GraphEntry {
  const double *poses;
  double *H, *b, *e;
  int64_t *inl;
  int32_t *corr;
  int accum;
  int resid;
  int fused;
  float kappa;
  int kind;
  int form;  // VGICP_FORM_SOURCE or VGICP_FORM_PAIR
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;  // factor set's replay counter at the last launch
};

// Captured graphs a factor set keeps; capturing one more drops the least
// recently replayed.
constexpr size_t kMaxGraphs = 8;

struct vgicp_factorset_s {
  int device = 0;
  int64_t n_factors = 0;
  int64_t n_tiles = 0;
  int64_t total_points = 0;
  int32_t n_poses = 0;
  int32_t tile_points = 0;
  // Blocks of a persistent grid (a multiple of 8), 0 for one block per tile.
  int32_t persist_blocks = 0;
  vgicp::FactorDesc *d_factors = nullptr;  // device
  // device [n_factors] relative-pose constants, rewritten by every round over
  // the whole tile table before its linearize launch (kFactorConstsBytes each)
  void *d_consts = nullptr;
  vgicp::Tile *d_tiles = nullptr;          // device
  double *d_partials = nullptr;            // device [n_tiles][kPartialStride]
  // Pair-form tile partials, [pair_capacity][kPairStride], allocated at the
  // first pair-form call.
  double *d_partials_pair = nullptr;
  int64_t pair_capacity = 0;
  int32_t form = VGICP_FORM_SOURCE;  // the form of VGICP_FORM_AUTO calls
  std::vector<vgicp::FactorDesc> h_factors;
  std::vector<int64_t> tile_order;  // factors in tile order (grouped by target map)
  std::vector<int32_t> h_src;       // source cloud of each factor
  int32_t layout = VGICP_LAYOUT_GROUPED;  // tile table layout (VGICP_LAYOUT_*)
  void *d_sorted = nullptr;  // device: ordered copies of the source clouds
  // Source points with a non-finite coordinate / covariance entry, counted
  // when the ordered copies were made.
  int64_t nonfinite_points = 0, nonfinite_covs = 0;
  int64_t tiles_capacity = 0;       // tiles d_tiles and d_partials have room for
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  // System assembly: contributions to each pose (CSR over poses, entries are
  // factor * 4 + side (0 = as pose i, 1 = as pose j) + 2 for a factor whose
  // two poses coincide, on its pose-i entry) and to each
  // unordered pose pair (CSR over pairs, entries factor * 2 + flip, flip 1
  // when the factor's (i, j) is the pair's (q, p)).
  std::vector<int32_t> h_pairs;   // [n_pairs][2]
  int64_t n_pairs = 0;
  int64_t *d_pose_off = nullptr, *d_pose_ent = nullptr;
  int64_t *d_pair_off = nullptr, *d_pair_ent = nullptr;
};
