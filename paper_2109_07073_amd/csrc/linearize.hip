// VGICP factor linearization, cost evaluation and overlap on gfx950.
//
// Paper: Sec. III-A, Eqs. (2)-(6) (Hessian factor of one matching-cost
// factor) and Sec. III-B, Eqs. (7)-(8) (overlap).  The sums of Eqs. (3), (5)
// and (6) are reduced without atomics: every workgroup tile writes one
// partial, and a second kernel adds a factor's partials in a fixed order.
//
// Per-point work is 3x3 algebra, not a dense contraction, so everything runs
// on the vector ALUs: FP32 per-point algebra with the residual in FP64, FP64
// per-factor sums.
//
// Source-frame form.  With T = T_j^-1 T_i = (R, t) and the right perturbation
// of T_i, A_k = R [[mu]x, -I], so A^T Omega A = J'^T Omega' J' with
// J' = [[mu]x, -I] and Omega' = R^T Omega R = (R^T C'_k R + C_k)^-1.  Each
// point therefore adds to a symmetric 6x6 (21 sums), a 6-vector and the cost:
// 28 sums instead of the 78 + 12 + 1 of the 12x12 system.  The remaining
// blocks follow exactly from B_k = -A_k Ad(T^-1):
//   H_ij = -H_ii Ad,  H_jj = Ad^T H_ii Ad,  b_j = -Ad^T b_i,
// which the reduce kernel applies once per factor in FP64.

#include <algorithm>

#include "vgicp_internal.hpp"

namespace vgicp {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------- poses
// T_j^-1 T_i in FP64 with a fixed evaluation order and no contraction, and
// exactly (I, 0) for bitwise-equal poses.  The FP32 rounding of this pose,
// scaled by the map's 1/r, drives the correspondence decision, so its order is
// part of the contract.
__device__ __forceinline__ void relative_pose64(const double *__restrict__ pi,
                                                const double *__restrict__ pj, double R[9],
                                                double t[3]) {
#pragma clang fp contract(off)
  bool same = true;
#pragma unroll
  for (int k = 0; k < 12; ++k) same &= (__double_as_longlong(pi[k]) == __double_as_longlong(pj[k]));
  if (same) {
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    t[0] = t[1] = t[2] = 0.0;
    return;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      R[3 * r + c] = (pj[r] * pi[c] + pj[3 + r] * pi[3 + c]) + pj[6 + r] * pi[6 + c];
  const double d0 = pi[9] - pj[9], d1 = pi[10] - pj[10], d2 = pi[11] - pj[11];
#pragma unroll
  for (int r = 0; r < 3; ++r) t[r] = (pj[r] * d0 + pj[3 + r] * d1) + pj[6 + r] * d2;
}

// The FP32 coordinates, in voxel units, that decide the correspondence of a
// point (the voxel holding T_j^-1 T_i mu, Sec. III-A): three fused
// multiply-adds per axis with the rotation and translation scaled by the
// map's fl32(1/r), each rounded once to FP32.
__device__ __forceinline__ void lookup_coords(const float S[9], const float u[3], float x,
                                              float y, float z, float v[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    v[r] = __builtin_fmaf(S[3 * r + 2], z,
                          __builtin_fmaf(S[3 * r + 1], y, __builtin_fmaf(S[3 * r], x, u[r])));
}

// The plain FP32 transform R mu + t (fixed order, no fused multiply-add),
// used only by the FP32 residual variant.
__device__ __forceinline__ void transform_fp32(const float R[9], const float t[3], float x,
                                               float y, float z, float q[3]) {
#pragma clang fp contract(off)
  q[0] = ((R[0] * x + R[1] * y) + R[2] * z) + t[0];
  q[1] = ((R[3] * x + R[4] * y) + R[5] * z) + t[1];
  q[2] = ((R[6] * x + R[7] * y) + R[8] * z) + t[2];
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x3 __attribute__((ext_vector_type(3)));

// ---------------------------------------------------------------- buffer loads
// Clouds and maps are read through raw buffer resources: a uniform base in
// scalar registers plus a 32-bit byte offset per lane (no 64-bit address
// arithmetic per lane), and a load at or past the resource's size returns
// zeros, so the coordinate prefetch past a tile's last point needs no clamp.
// The size limits of clouds and maps keep every offset below 2^32.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // 32-bit data format, no swizzle
constexpr int kNT = 2;                  // nontemporal: streamed once

__device__ __forceinline__ Rsrc make_rsrc(const void *p, uint64_t bytes) {
  const uint32_t num = bytes < 0xffffffffull ? uint32_t(bytes) : 0xffffffffu;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, int(num), kRsrcWord3);
}

template <int AUX = 0>
__device__ __forceinline__ float ld_f32(Rsrc r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(off), 0, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ f32x3 ld_f32x3(Rsrc r, uint32_t off) {
  return __builtin_bit_cast(f32x3, __builtin_amdgcn_raw_buffer_load_b96(r, int(off), 0, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ f32x4 ld_f32x4(Rsrc r, uint32_t off) {
  return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, int(off), 0, AUX));
}

// The coordinates of one tile, points [begin, end) of a source copy stored
// point by point ([n][3]): one 12-byte load per lane and pass.  The prefetch
// past the tile's end reads zeros without touching memory (it would otherwise
// fetch the next tile's lines).
struct CloudRsrc {
  Rsrc p;
};

__device__ __forceinline__ CloudRsrc tile_rsrc(const float *xyz, uint32_t begin, uint32_t end) {
  return {make_rsrc(xyz + 3ull * begin, 12ull * (end - begin))};
}

// Point `i` of the tile (counted from its first point).
__device__ __forceinline__ void load_xyz(const CloudRsrc &c, uint32_t i, float p[3]) {
  const f32x3 v = ld_f32x3<kNT>(c.p, i * 12u);
  p[0] = v.x, p[1] = v.y, p[2] = v.z;
}

// Brick key halves, home record and bit of the voxel holding the point with
// lookup coordinates v.  Each coordinate is clamped to [-2^20 - 4, 2^20] (NaN
// goes to the low end), so a point outside the key range names a brick that
// no map holds.
struct VoxelKey {
  uint32_t klo, khi;  // packed brick key
  uint32_t h;         // home record
  uint32_t up;        // 63 - the voxel's bit in the brick's occupancy mask
};

// floor(x) as an integer, one v_cvt_flr_i32_f32 (the compiler emits a floor
// and a conversion); x is finite and within [-2^20 - 4, 2^20] here.
__device__ __forceinline__ int32_t floor_i32(float x) {
  int32_t k;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(k) : "v"(x));
  return k;
}

// Table of 63 - brick_bit over the low two key bits per axis, entry
// 16 (kx & 3) + 4 (ky & 3) + (kz & 3): the index takes five instructions
// against ten for the interleave.  `up_table_fill` writes it into a block's
// LDS (the caller synchronizes before the first lookup).
constexpr int kUpTable = 64;

__device__ __forceinline__ void up_table_fill(uint8_t *t) {
  const uint32_t i = threadIdx.x;
  if (i < uint32_t(kUpTable))
    t[i] = uint8_t(brick_bit(int32_t(i >> 4), int32_t(i >> 2) & 3, int32_t(i) & 3) ^ 63u);
}

// With kTable the voxel's bit comes from the table `up` in LDS, else it is
// computed.
template <bool kTable = false>
__device__ __forceinline__ VoxelKey voxel_key(const float v[3], uint32_t log2cap,
                                              const uint8_t *up = nullptr) {
  const float vx = fminf(fmaxf(v[0], kClampLoF), kClampHiF);
  const float vy = fminf(fmaxf(v[1], kClampLoF), kClampHiF);
  const float vz = fminf(fmaxf(v[2], kClampLoF), kClampHiF);
  const int32_t kx = floor_i32(vx), ky = floor_i32(vy), kz = floor_i32(vz);
  const uint32_t fx = brick_field(kx), fy = brick_field(ky), fz = brick_field(kz);
  VoxelKey r;
  r.klo = (fy << kBrickBits) | fz;
  r.khi = (fx << (2 * kBrickBits - 32)) | (fy >> (32 - kBrickBits));
  if constexpr (kTable) {
    const uint32_t i = (uint32_t(kx & 3) << 4) | (uint32_t(ky & 3) << 2) | uint32_t(kz & 3);
    r.up = up[i];
  } else {
    r.up = brick_bit(kx, ky, kz) ^ 63u;
  }
  r.h = brick_slot(fx, fy, fz, log2cap);
  return r;
}

// A brick record as loaded: key and mask (one 16-byte load) and the index of
// the brick's first voxel.
struct RecordLoad {
  f32x4 km;
  uint32_t base;
};

__device__ __forceinline__ RecordLoad load_record(Rsrc rb, uint32_t h) {
  RecordLoad r;
  r.km = ld_f32x4(rb, h << 5);
  r.base = __builtin_bit_cast(uint32_t, ld_f32(rb, (h << 5) + 16u));
  return r;
}

// Byte mask of the occupancy word of record h: the word is at byte
// (h >> 3) & occ_word_mask(occ_mask) of the bitset, ((h & occ_mask) >> 5) * 4.
__device__ __forceinline__ uint32_t occ_word_mask(uint32_t occ_mask) {
  uint32_t m = (occ_mask >> 3) & ~3u;
  // opaque to the optimizer, which would otherwise expand (h >> 3) & m back
  // into three operations per lookup
  asm("" : "+s"(m));
  return m;
}

// Whether the table's occupancy bitset (staged in LDS) has record h's bit set;
// wmask = occ_word_mask(occ_mask).
__device__ __forceinline__ bool home_occupied(const uint32_t *occ, uint32_t wmask, uint32_t h) {
  const uint32_t w = *reinterpret_cast<const uint32_t *>(
      reinterpret_cast<const char *>(occ) + ((h >> 3) & wmask));
  return __builtin_amdgcn_ubfe(w, h, 1u) != 0u;  // bit h mod 32
}

// The home record of a lookup, read only when its bit is set: otherwise the
// offset lies past the table, so the load returns zeros without a memory
// request (for a table of the largest size it reads the last record, which
// the caller ignores).
__device__ __forceinline__ RecordLoad load_home(Rsrc rb, uint32_t h, bool occupied) {
  const uint32_t off = occupied ? (h << 5) : 0xffffffe0u;
  RecordLoad r;
  r.km = ld_f32x4(rb, off);
  r.base = __builtin_bit_cast(uint32_t, ld_f32(rb, off + 16u));
  return r;
}

__device__ __forceinline__ uint64_t u64_of(float lo, float hi) {
  return (uint64_t(__builtin_bit_cast(uint32_t, hi)) << 32) | __builtin_bit_cast(uint32_t, lo);
}

// Voxel index of the point, or -1: the home record (unless its occupancy bit
// is clear), or the records after it at the same position of the following
// lines up to the first free one (linear probing), must hold the brick,
// and its mask the voxel's bit.  Probing is rare (a home record of another
// brick), so it runs behind one wave-uniform branch and the common path has
// no divergent control flow.  At most capacity / 4 records are visited.
__device__ __forceinline__ int find_voxel(Rsrc rb, uint32_t log2cap, const VoxelKey &vk,
                                          const RecordLoad &home, bool occupied) {
  const uint64_t key = (uint64_t(vk.khi) << 32) | vk.klo;
  uint64_t rkey = u64_of(home.km.x, home.km.y);
  uint64_t mask = u64_of(home.km.z, home.km.w);
  uint32_t base = home.base;
  const bool probe = occupied && rkey != key && rkey != kEmptyKey;
  if (__builtin_amdgcn_ballot_w64(probe) != 0) {
    if (probe) {
      const uint32_t cm = (1u << log2cap) - 1u;
      uint32_t h = vk.h;
      for (uint32_t p = 0; p < (cm >> 2); ++p) {
        h = (h + kProbeStep) & cm;
        const RecordLoad r = load_record(rb, h);
        const uint64_t k2 = u64_of(r.km.x, r.km.y);
        if (k2 == key) {
          rkey = key;
          mask = u64_of(r.km.z, r.km.w);
          base = r.base;
          break;
        }
        if (k2 == kEmptyKey) break;
      }
    }
    // leave no load of this path in flight, so the common path's waits
    // stay exact
    __builtin_amdgcn_s_waitcnt(0);
  }
  // the voxel's bit moved to the top: set for a hit, and the bits of the mask
  // at and below it count the voxel and the brick's voxels before it
  const uint64_t top = mask << vk.up;
  if (!occupied || rkey != key || int64_t(top) >= 0) return -1;
  return int(base + uint32_t(__popcll(top)) - 1u);
}

// ---------------------------------------------------------------- sums
// Wave64 sums with DPP row operations (VALU only, no LDS traffic): pairs,
// quads, half rows, rows, then row broadcasts 15 and 31.  The total ends in
// lane 63.  Lanes of rows a broadcast does not write keep `old` = 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(v)));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL, ROW_MASK>(int(b & 0xffffffffll));
  const int hi = dpp_i<CTRL, ROW_MASK>(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}

#define VGICP_DPP_STEPS(F, v)      \
  v += F<0xb1>(v);                  \
  v += F<0x4e>(v);                  \
  v += F<0x141>(v);                 \
  v += F<0x140>(v);                 \
  v += F<0x142, 0xa>(v);            \
  v += F<0x143, 0xc>(v);

__device__ __forceinline__ float wave_sum(float v) {
  VGICP_DPP_STEPS(dpp_f, v)
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  VGICP_DPP_STEPS(dpp_d, v)
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
  VGICP_DPP_STEPS(dpp_i, v)
  return v;
}
constexpr int kLastLane = 63;

template <int ACC, int N>
struct Sums;

template <int N>
struct Sums<VGICP_ACC_F32, N> {
  float v[N];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0.f;
  }
  __device__ __forceinline__ void add(int i, float x) { v[i] += x; }
  __device__ void wave_reduce() {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  }
  __device__ void store(float *lds, int wave) const {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[wave * N + i] = v[i];
  }
  // The wave's sums into lds[wave * N + i] (the wave's hit ring, `ring`, is
  // free at this point; these forms do not use it).
  template <typename T>
  __device__ void reduce_to(T *lds, int wave, uint32_t lane, float *ring) {
    (void)ring;
    wave_reduce();
    if (lane == kLastLane) store(lds, wave);
  }
  using lds_t = float;
  __device__ static double finish(const float *lds, int i) {
    float s = lds[i];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += lds[w * N + i];
    return double(s);
  }
};

template <int N>
struct Sums<VGICP_ACC_F64, N> {
  double v[N];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0.0;
  }
  __device__ __forceinline__ void add(int i, float x) { v[i] += double(x); }
  __device__ void wave_reduce() {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  }
  __device__ void store(double *lds, int wave) const {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[wave * N + i] = v[i];
  }
  // The wave's sums into lds[wave * N + i] (the wave's hit ring, `ring`, is
  // free at this point; these forms do not use it).
  template <typename T>
  __device__ void reduce_to(T *lds, int wave, uint32_t lane, float *ring) {
    (void)ring;
    wave_reduce();
    if (lane == kLastLane) store(lds, wave);
  }
  using lds_t = double;
  __device__ static double finish(const double *lds, int i) {
    double s = lds[i];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += lds[w * N + i];
    return s;
  }
};

// Knuth's two-sum: a + b = s + err exactly (s = fl(a + b)).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &err) {
#pragma clang fp contract(off)
  s = a + b;
  const float bp = s - a;
  err = (a - (s - bp)) + (b - bp);
}

// Source-frame residual r = R^T (m - (R mu + t)) = R^T (m - t) - mu, in FP64
// from the FP32 point and voxel mean and the FP64 relative pose, rounded once
// to FP32.  FP64 fused multiply-adds issue at the unpacked FP32 rate on
// gfx950, so this costs about as much as an FP32 transform and rotation and is
// accurate to the rounding of the residual itself.
__device__ __forceinline__ void residual64(const double R[9], const double t[3], float x,
                                           float y, float z, const float m[3], float r[3]) {
  const double d0 = double(m[0]) - t[0], d1 = double(m[1]) - t[1], d2 = double(m[2]) - t[2];
  const double p[3] = {x, y, z};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double q = __builtin_fma(R[6 + c], d2, __builtin_fma(R[3 + c], d1, R[c] * d0));
    r[c] = float(q - p[c]);
  }
}

// Compensated FP32: a lane adds its few terms of a tile (about 36 points, 40 %
// of them hits, at the largest tile) in plain FP32, like VGICP_ACC_F32, so it
// keeps the same registers and occupancy; the reduction over the 64 lanes of
// a wave carries a (sum, error) pair through every DPP step with two-sum, and
// waves and tiles are then added in FP64.
template <int N>
struct Sums<VGICP_ACC_F32_COMP, N> {
  float v[N];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0.f;
  }
  __device__ __forceinline__ void add(int i, float x) { v[i] += x; }
  // Each DPP step adds a partner's (sum, compensation) pair with two-sum.
  template <int CTRL, int ROW_MASK = 0xf>
  __device__ __forceinline__ static void step(float &v, float &c) {
    const float ov = dpp_f<CTRL, ROW_MASK>(v);
    const float oc = dpp_f<CTRL, ROW_MASK>(c);
    float s, err;
    two_sum(v, ov, s, err);
    v = s;
    c = c + oc + err;
  }
  __device__ void wave_reduce() {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      float c = 0.f;
      step<0xb1>(v[i], c);
      step<0x4e>(v[i], c);
      step<0x141>(v[i], c);
      step<0x140>(v[i], c);
      step<0x142, 0xa>(v[i], c);
      step<0x143, 0xc>(v[i], c);
      wide[i] = double(v[i]) + double(c);
    }
  }
  double wide[N];  // the wave's (sum + compensation) in FP64, after wave_reduce
  __device__ void store(double *lds, int wave) const {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[wave * N + i] = wide[i];
  }
  // The wave's (sum + compensation) values, in FP64, into lds[wave * N + i].
  // A single sum goes through the DPP tree above.  The 28 sums of a
  // linearization are transposed through the wave's hit ring (free at the end
  // of a tile), 14 at a time as in the FP64-carried form: four lanes per sum
  // each add 16 values of its column with two-sum, and two quad DPP steps add
  // the four (sum, compensation) pairs with two-sum.
  // sums per pass: 14 for the 28 source-frame sums, 13 for the pair form's 91
  static constexpr int kGroup = N % 14 == 0 ? 14 : N % 13 == 0 ? 13 : 0;
  static constexpr int kStride = kGroup + 1;
  template <typename T>
  __device__ void reduce_to(T *lds, int wave, uint32_t lane, float *ring) {
    if constexpr (kGroup == 0) {
      (void)ring;
      wave_reduce();
      if (lane == kLastLane) store(lds, wave);
    } else {
      const uint32_t c = lane >> 2, q = lane & 3;
#pragma unroll
      for (int g = 0; g < N; g += kGroup) {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kGroup; ++i) ring[lane * kStride + i] = v[g + i];
        __builtin_amdgcn_wave_barrier();
        float sum = 0.f, comp = 0.f;
        if (c < uint32_t(kGroup)) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            float s, err;
            two_sum(sum, ring[(4 * r + q) * kStride + c], s, err);
            sum = s;
            comp += err;
          }
        }
        step<0xb1>(sum, comp);  // quad lanes (1, 0, 3, 2)
        step<0x4e>(sum, comp);  // quad lanes (2, 3, 0, 1)
        if (c < uint32_t(kGroup) && q == 0) lds[wave * N + g + int(c)] = double(sum) + double(comp);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  using lds_t = double;
  __device__ static double finish(const double *lds, int i) {
    double s = lds[i];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += lds[w * N + i];
    return s;
  }
};

// FP32 per lane, FP64 beyond: a lane adds its few terms of a tile in FP32 (the
// registers and occupancy of VGICP_ACC_F32); each lane sum is then widened
// exactly to FP64, and the sum over the wave's lanes, the waves and the tiles
// are FP64.
template <int N>
struct Sums<VGICP_ACC_MIXED, N> {
  float v[N];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0.f;
  }
  __device__ __forceinline__ void add(int i, float x) { v[i] += x; }
  // The wave's sums in FP64 into lds[wave * N + i].  A single sum goes through
  // the DPP tree.  The 28 sums of a linearization are transposed through the
  // wave's hit ring instead (free at the end of a tile; 5,120 bytes): 14 sums
  // at a time, every lane writes its 14 FP32 sums as one row (stride 15 words),
  // then four lanes per sum each add a quarter of that sum's column, 16 values,
  // in FP64 (exact for FP32 inputs of like magnitude), and a quad DPP step
  // pair adds the four quarters: about 80 VALU instructions for all 28 sums
  // against 530 for 28 DPP trees in FP64.
  // sums per pass: 14 for the 28 source-frame sums, 13 for the pair form's 91
  static constexpr int kGroup = N % 14 == 0 ? 14 : N % 13 == 0 ? 13 : 0;
  static constexpr int kStride = kGroup + 1;
  template <typename T>
  __device__ void reduce_to(T *lds, int wave, uint32_t lane, float *ring) {
    if constexpr (kGroup == 0) {
      (void)ring;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double w = wave_sum(double(v[i]));
        if (lane == kLastLane) lds[wave * N + i] = w;
      }
    } else {
      const uint32_t c = lane >> 2, q = lane & 3;
#pragma unroll
      for (int g = 0; g < N; g += kGroup) {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kGroup; ++i) ring[lane * kStride + i] = v[g + i];
        __builtin_amdgcn_wave_barrier();
        double sum = 0.0;
        if (c < uint32_t(kGroup)) {
#pragma unroll
          for (int r = 0; r < 16; ++r) sum += double(ring[(4 * r + q) * kStride + c]);
        }
        sum += dpp_d<0xb1>(sum);  // quad lanes (1, 0, 3, 2)
        sum += dpp_d<0x4e>(sum);  // quad lanes (2, 3, 0, 1)
        if (c < uint32_t(kGroup) && q == 0) lds[wave * N + g + int(c)] = sum;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  using lds_t = double;
  __device__ static double finish(const double *lds, int i) {
    double s = lds[i];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += lds[w * N + i];
    return s;
  }
};

// ---------------------------------------------------------------- factor constants
struct FactorConsts {
  float S[9];     // fl32(s R): lookup coordinates
  float u[3];     // fl32(s t): lookup coordinates
  float R[9];     // fl32(R): per-point algebra and the FP32 residual
  float t[3];     // fl32(t): FP32 residual
  double R64[9];  // R itself: FP64 residual and FP64 fused covariance
  double t64[3];  // t itself: FP64 residual
};
static_assert(sizeof(FactorConsts) == kFactorConstsBytes, "the factor set's constant table");

__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}

// ---------------------------------------------------------------- per point
// (R^T S R + c)^-1 (for S = C', c = C the source-frame weight Omega') formed
// and inverted in FP64 from the FP32 covariances and the FP64 rotation R,
// rounded to FP32.  Used where forming the fused covariance in FP32 already
// loses its small eigenvalue.  Returns false when it is not positive definite.
__device__ __forceinline__ bool fused_information_fp64(const double R[9], const float S[6],
                                                    const float c[6], float o[6]) {
  const double s0 = S[0], s1 = S[1], s2 = S[2], s3 = S[3], s4 = S[4], s5 = S[5];
  double W[9];
#pragma unroll
  for (int col = 0; col < 3; ++col) {
    const double r0 = R[col], r1 = R[3 + col], r2 = R[6 + col];
    W[col] = s0 * r0 + s1 * r1 + s2 * r2;
    W[3 + col] = s1 * r0 + s3 * r1 + s4 * r2;
    W[6 + col] = s2 * r0 + s4 * r1 + s5 * r2;
  }
  auto f = [&](int a, int b, double cc) {
    return R[a] * W[b] + R[3 + a] * W[3 + b] + R[6 + a] * W[6 + b] + cc;
  };
  const double f00 = f(0, 0, c[0]), f01 = f(0, 1, c[1]), f02 = f(0, 2, c[2]);
  const double f11 = f(1, 1, c[3]), f12 = f(1, 2, c[4]), f22 = f(2, 2, c[5]);
  const double a00 = f11 * f22 - f12 * f12, a01 = f02 * f12 - f01 * f22;
  const double a02 = f01 * f12 - f02 * f11, a11 = f00 * f22 - f02 * f02;
  const double a12 = f01 * f02 - f00 * f12, a22 = f00 * f11 - f01 * f01;
  const double det = f00 * a00 + f01 * a01 + f02 * a02;
  // leading minors f00, a22 (of the upper 2x2) and det positive; a finite
  // det also excludes every infinite entry (each one makes det infinite or
  // NaN, or a22 negative), and NaN fails every comparison
  if (!(f00 > 0.0 && a22 > 0.0 && det > 0.0 && det < __builtin_huge_val())) return false;
  // hardware reciprocal estimate refined by two Newton steps (det is far
  // from the FP64 subnormal range: F' comes from FP32 entries)
  double inv = __builtin_amdgcn_rcp(det);
  inv = __builtin_fma(__builtin_fma(-det, inv, 1.0), inv, inv);
  inv = __builtin_fma(__builtin_fma(-det, inv, 1.0), inv, inv);
  o[0] = float(a00 * inv);
  o[1] = float(a01 * inv);
  o[2] = float(a02 * inv);
  o[3] = float(a11 * inv);
  o[4] = float(a12 * inv);
  o[5] = float(a22 * inv);
  return true;
}

// How the fused information Omega' = F'^-1 of a hit is formed:
//   kFuse64:   F', its adjugate and determinant in FP64 for every hit (F' of
//              a point on a surface has a condition number near 1e3 with
//              covariances regularized to (1, 1, 1e-3), so forming it in FP32
//              already costs about 1e3 ulp in the normal direction);
//   kFuse32:   all in FP32;
//   kFuseGate: FP32, and FP64 for hits whose FP32 F' is not positive definite
//              or has a condition estimate trace^3 / (27 det) above kappa.
constexpr int kFuse32 = 0;
constexpr int kFuseGate = 1;
constexpr int kFuse64 = 2;

// Adds one correspondence.  k holds the FP32 relative rotation (and its FP64
// value), (mx, my, mz) is the source point, c its covariance, r its residual
// R^T (mu' - T mu) in the source frame, S the voxel covariance.  With LIN the
// 21 + 6 source-frame Hessian/gradient sums and the cost are added; without
// it only the cost.  FUSE selects how Omega' is formed (above); with
// kFuseGate `nwide` counts the hits that took the FP64 path.  Returns false,
// adding nothing, for a hit whose fused covariance is not positive definite.
// The weight Omega = (R^T A R + B)^-1 of a correspondence (upper triangle
// xx xy xz yy yz zz), formed as FUSE selects (above): R^T C' R + C with the
// relative rotation R, the voxel covariance A = C' and the point covariance
// B = C is the source-frame fused covariance F'; passing R^T, A = C and B = C'
// gives the target-frame F = C' + R C R^T of Eq. (2).  R64 is R in FP64.
// With kFuseGate `nwide` counts the FP64 formations.  Returns false, leaving
// o unset, when the fused covariance is not positive definite.
template <int FUSE>
__device__ __forceinline__ bool fused_weight(const float R[9], const double R64[9],
                                             const float S[6], const float c[6], float kappa,
                                             uint32_t &nwide, float o[6]) {
#pragma clang fp contract(off)
#define FMA __builtin_fmaf
  float o00, o01, o02, o11, o12, o22;
  if constexpr (FUSE == kFuse64) {
    float w[6];
    if (!fused_information_fp64(R64, S, c, w)) return false;  // not positive definite
    o00 = w[0], o01 = w[1], o02 = w[2], o11 = w[3], o12 = w[4], o22 = w[5];
  } else {
    // W = S R, then F = R^T W + c (symmetric, upper triangle)
    const float W00 = FMA(S[2], R[6], FMA(S[1], R[3], S[0] * R[0]));
    const float W01 = FMA(S[2], R[7], FMA(S[1], R[4], S[0] * R[1]));
    const float W02 = FMA(S[2], R[8], FMA(S[1], R[5], S[0] * R[2]));
    const float W10 = FMA(S[4], R[6], FMA(S[3], R[3], S[1] * R[0]));
    const float W11 = FMA(S[4], R[7], FMA(S[3], R[4], S[1] * R[1]));
    const float W12 = FMA(S[4], R[8], FMA(S[3], R[5], S[1] * R[2]));
    const float W20 = FMA(S[5], R[6], FMA(S[4], R[3], S[2] * R[0]));
    const float W21 = FMA(S[5], R[7], FMA(S[4], R[4], S[2] * R[1]));
    const float W22 = FMA(S[5], R[8], FMA(S[4], R[5], S[2] * R[2]));
    const float f00 = FMA(R[6], W20, FMA(R[3], W10, FMA(R[0], W00, c[0])));
    const float f01 = FMA(R[6], W21, FMA(R[3], W11, FMA(R[0], W01, c[1])));
    const float f02 = FMA(R[6], W22, FMA(R[3], W12, FMA(R[0], W02, c[2])));
    const float f11 = FMA(R[7], W21, FMA(R[4], W11, FMA(R[1], W01, c[3])));
    const float f12 = FMA(R[7], W22, FMA(R[4], W12, FMA(R[1], W02, c[4])));
    const float f22 = FMA(R[8], W22, FMA(R[5], W12, FMA(R[2], W02, c[5])));
    // Omega = F^-1 by the adjugate
    const float a00 = FMA(f11, f22, -(f12 * f12));
    const float a01 = FMA(f02, f12, -(f01 * f22));
    const float a02 = FMA(f01, f12, -(f02 * f11));
    const float a11 = FMA(f00, f22, -(f02 * f02));
    const float a12 = FMA(f01, f02, -(f00 * f12));
    const float a22 = FMA(f00, f11, -(f01 * f01));
    const float det = FMA(f02, a02, FMA(f01, a01, f00 * a00));
    // positive definite: leading minors f00, a22 (upper 2x2) and det positive.
    // An infinite entry makes det infinite or NaN (or a22 negative), so a
    // finite det also excludes those; NaN fails every comparison.
    const bool pd32 = (f00 > 0.f) & (a22 > 0.f) & (det > 0.f) & (det < __builtin_huge_valf());
    bool wide = false;
    if constexpr (FUSE == kFuseGate) {
      const float tr = (f00 + f11) + f22;
      wide = !pd32 || (tr * tr * tr > (27.0f * kappa) * det);
    }
    if (wide) {
      ++nwide;
      float w[6];
      if (!fused_information_fp64(R64, S, c, w)) return false;  // not positive definite
      o00 = w[0], o01 = w[1], o02 = w[2], o11 = w[3], o12 = w[4], o22 = w[5];
    } else {
      if (!pd32) return false;  // not positive definite
      // hardware reciprocal refined by one Newton step (within an ulp or so;
      // det > 0 here and far above the FP32 subnormal range for these inputs)
      const float r0i = __builtin_amdgcn_rcpf(det);
      const float inv = FMA(FMA(-det, r0i, 1.0f), r0i, r0i);
      o00 = a00 * inv, o01 = a01 * inv, o02 = a02 * inv;
      o11 = a11 * inv, o12 = a12 * inv, o22 = a22 * inv;
    }
  }
  o[0] = o00, o[1] = o01, o[2] = o02, o[3] = o11, o[4] = o12, o[5] = o22;
#undef FMA
  return true;
}

template <bool LIN, int FUSE, typename SumsT>
__device__ __forceinline__ bool add_correspondence(SumsT &acc, const FactorConsts &k,
                                                   float kappa, float mx, float my, float mz,
                                                   const float c[6], const float r[3],
                                                   const float S[6], uint32_t &nwide) {
  // Contraction is off and every fused multiply-add is explicit, so the cost
  // comes out bit-identical in the linearization and the cost-only kernels.
#pragma clang fp contract(off)
#define FMA __builtin_fmaf
  const float r0 = r[0], r1 = r[1], r2 = r[2];
  float o[6];
  if (!fused_weight<FUSE>(k.R, k.R64, S, c, kappa, nwide, o)) return false;  // not PD
  const float o00 = o[0], o01 = o[1], o02 = o[2], o11 = o[3], o12 = o[4], o22 = o[5];
  // g = Omega' r
  const float g0 = FMA(o02, r2, FMA(o01, r1, o00 * r0));
  const float g1 = FMA(o12, r2, FMA(o11, r1, o01 * r0));
  const float g2 = FMA(o22, r2, FMA(o12, r1, o02 * r0));
  acc.add(LIN ? 27 : 0, FMA(r2, g2, FMA(r1, g1, r0 * g0)));
  if constexpr (LIN) {
    // M = [mu]x Omega' (column c = mu x Omega'_c): the (omega, rho) block
    const float M00 = FMA(my, o02, -(mz * o01)), M10 = FMA(mz, o00, -(mx * o02));
    const float M20 = FMA(mx, o01, -(my * o00));
    const float M01 = FMA(my, o12, -(mz * o11)), M11 = FMA(mz, o01, -(mx * o12));
    const float M21 = FMA(mx, o11, -(my * o01));
    const float M02 = FMA(my, o22, -(mz * o12)), M12 = FMA(mz, o02, -(mx * o22));
    const float M22 = FMA(mx, o12, -(my * o02));
    // (omega, omega) block [mu]x^T Omega' [mu]x, row r = mu x (row r of M)
    acc.add(0, FMA(my, M02, -(mz * M01)));
    acc.add(1, FMA(mz, M00, -(mx * M02)));
    acc.add(2, FMA(mx, M01, -(my * M00)));
    acc.add(3, M00);
    acc.add(4, M01);
    acc.add(5, M02);
    acc.add(6, FMA(mz, M10, -(mx * M12)));
    acc.add(7, FMA(mx, M11, -(my * M10)));
    acc.add(8, M10);
    acc.add(9, M11);
    acc.add(10, M12);
    acc.add(11, FMA(mx, M21, -(my * M20)));
    acc.add(12, M20);
    acc.add(13, M21);
    acc.add(14, M22);
    acc.add(15, o00);
    acc.add(16, o01);
    acc.add(17, o02);
    acc.add(18, o11);
    acc.add(19, o12);
    acc.add(20, o22);
    // gradient J'^T Omega' r = (g x mu, -g)
    acc.add(21, FMA(g1, mz, -(g2 * my)));
    acc.add(22, FMA(g2, mx, -(g0 * mz)));
    acc.add(23, FMA(g0, my, -(g1 * mx)));
    acc.add(24, -g0);
    acc.add(25, -g1);
    acc.add(26, -g2);
  }
#undef FMA
  return true;
}

// ---------------------------------------------------------------- pair form
// The per-correspondence Hessian factor of Eqs. (5)-(6) in the target frame,
// accumulated term by term: with q = R mu + t, the residual e = mu' - q, the
// weight Omega = (C' + R C R^T)^-1 of Eq. (2) and the Jacobians under right
// perturbations xi = (omega, rho) of T_i and T_j,
//   A = de/dxi_i = [R [mu]x, -R],   B = de/dxi_j = [-[q]x, I],
// a correspondence adds J^T Omega J to the 12 x 12 H (J = [A, B]; its 78
// upper-triangle entries, row-major), J^T Omega e to b (12) and e^T Omega e
// to the cost: 91 sums.  Intermediates: N = Omega R, P = Omega A =
// [N [mu]x, -N], K = R [mu]x, Q = Omega [q]x, g = Omega e; then
//   H_ii = [[K^T N [mu]x, -K^T N], [., R^T N]],
//   H_ij = P^T B = [P^T (-[q]x), P^T],
//   H_jj = [[-[q]x Q, -Q^T], [., Omega]],
//   b = (K^T g, -R^T g, q x g, g).
// Index of H entry (r, c), r <= c, in the row-major upper triangle of 12 x 12.
__host__ __device__ constexpr int pair_index(int r, int c) {
  return r * 12 - (r * (r - 1)) / 2 + (c - r);
}
static_assert(pair_index(11, 11) == 77, "78 upper-triangle entries");

// Target-frame residual and transformed point: q = R mu + t and e = m - q in
// FP64 from the FP32 point and voxel mean, each rounded once to FP32.
__device__ __forceinline__ void residual64_target(const double R[9], const double t[3], float x,
                                                  float y, float z, const float m[3], float e[3],
                                                  float q[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double qq = __builtin_fma(R[3 * r + 2], double(z),
                                    __builtin_fma(R[3 * r + 1], double(y),
                                                  __builtin_fma(R[3 * r], double(x), t[r])));
    q[r] = float(qq);
    e[r] = float(double(m[r]) - qq);
  }
}

// Adds one correspondence in the pair form: (mx, my, mz) is the source point,
// c its covariance, e and q from residual64_target (or the FP32 transform),
// S the voxel covariance.  Returns false, adding nothing, when the fused
// covariance is not positive definite.
template <int FUSE, typename SumsT>
__device__ __forceinline__ bool add_pair_terms(SumsT &acc, const FactorConsts &k, float kappa,
                                               float mx, float my, float mz, const float c[6],
                                               const float e[3], const float q[3],
                                               const float S[6], uint32_t &nwide) {
#pragma clang fp contract(off)
#define FMA __builtin_fmaf
  const float *R = k.R;
  // F = (R^T)^T C (R^T) + C' with the transposed rotation
  const float RT[9] = {R[0], R[3], R[6], R[1], R[4], R[7], R[2], R[5], R[8]};
  const double RT64[9] = {k.R64[0], k.R64[3], k.R64[6], k.R64[1], k.R64[4],
                          k.R64[7], k.R64[2], k.R64[5], k.R64[8]};
  float w[6];
  if (!fused_weight<FUSE>(RT, RT64, c, S, kappa, nwide, w)) return false;  // not PD
  const float O[9] = {w[0], w[1], w[2], w[1], w[3], w[4], w[2], w[4], w[5]};
  float N[9];  // Omega R
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      N[3 * r + cc] = FMA(O[3 * r + 2], R[6 + cc], FMA(O[3 * r + 1], R[3 + cc], O[3 * r] * R[cc]));
  // X [v]x for a 3 x 3 X: column 0 = vz X_1 - vy X_2, 1 = vx X_2 - vz X_0,
  // 2 = vy X_0 - vx X_1 (X_c: column c)
  auto cross_cols = [&](const float X[9], float vx, float vy, float vz, float Y[9]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float x0 = X[3 * r], x1 = X[3 * r + 1], x2 = X[3 * r + 2];
      Y[3 * r] = FMA(vz, x1, -(vy * x2));
      Y[3 * r + 1] = FMA(vx, x2, -(vz * x0));
      Y[3 * r + 2] = FMA(vy, x0, -(vx * x1));
    }
  };
  float Pw[9], K[9], Q[9];
  cross_cols(N, mx, my, mz, Pw);  // Omega R [mu]x
  cross_cols(R, mx, my, mz, K);   // R [mu]x
  cross_cols(O, q[0], q[1], q[2], Q);  // Omega [q]x
  // column a of P = Omega A (a < 3: Pw, else -N)
  auto P = [&](int r, int a) { return a < 3 ? Pw[3 * r + a] : -N[3 * r + a - 3]; };
  auto dot3 = [&](float a0, float a1, float a2, float b0, float b1, float b2) {
    return FMA(a2, b2, FMA(a1, b1, a0 * b0));
  };
  // H_ii: A^T P, with A's columns (K, -R)
  auto A = [&](int r, int a) { return a < 3 ? K[3 * r + a] : -R[3 * r + a - 3]; };
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b2 = a; b2 < 6; ++b2)
      acc.add(pair_index(a, b2), dot3(A(0, a), A(1, a), A(2, a), P(0, b2), P(1, b2), P(2, b2)));
  // H_ij = [P^T (-[q]x), P^T]
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const float p0 = P(0, a), p1 = P(1, a), p2 = P(2, a);
    acc.add(pair_index(a, 6), FMA(p2, q[1], -(p1 * q[2])));
    acc.add(pair_index(a, 7), FMA(p0, q[2], -(p2 * q[0])));
    acc.add(pair_index(a, 8), FMA(p1, q[0], -(p0 * q[1])));
    acc.add(pair_index(a, 9), p0);
    acc.add(pair_index(a, 10), p1);
    acc.add(pair_index(a, 11), p2);
  }
  // H_jj = [[-[q]x Q, -Q^T], [., Omega]]
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const float q0 = Q[cc], q1 = Q[3 + cc], q2 = Q[6 + cc];  // column cc of Q
    const float t0 = FMA(q[2], q1, -(q[1] * q2));
    const float t1 = FMA(q[0], q2, -(q[2] * q0));
    const float t2 = FMA(q[1], q0, -(q[0] * q1));
    acc.add(pair_index(6, 6 + cc), t0);
    if (cc >= 1) acc.add(pair_index(7, 6 + cc), t1);
    if (cc >= 2) acc.add(pair_index(8, 6 + cc), t2);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc.add(pair_index(6 + r, 9 + cc), -Q[3 * cc + r]);
  acc.add(pair_index(9, 9), O[0]);
  acc.add(pair_index(9, 10), O[1]);
  acc.add(pair_index(9, 11), O[2]);
  acc.add(pair_index(10, 10), O[4]);
  acc.add(pair_index(10, 11), O[5]);
  acc.add(pair_index(11, 11), O[8]);
  // b and the cost
  const float g0 = dot3(O[0], O[1], O[2], e[0], e[1], e[2]);
  const float g1 = dot3(O[3], O[4], O[5], e[0], e[1], e[2]);
  const float g2 = dot3(O[6], O[7], O[8], e[0], e[1], e[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc.add(78 + a, dot3(K[a], K[3 + a], K[6 + a], g0, g1, g2));
    acc.add(81 + a, -dot3(R[a], R[3 + a], R[6 + a], g0, g1, g2));
  }
  acc.add(84, FMA(q[1], g2, -(q[2] * g1)));
  acc.add(85, FMA(q[2], g0, -(q[0] * g2)));
  acc.add(86, FMA(q[0], g1, -(q[1] * g0)));
  acc.add(87, g0);
  acc.add(88, g1);
  acc.add(89, g2);
  acc.add(90, dot3(e[0], e[1], e[2], g0, g1, g2));
#undef FMA
  return true;
}

// ---------------------------------------------------------------- tiles
// The constants of factor fd at `poses`, computed by this lane.
__device__ __forceinline__ FactorConsts factor_consts_lane(const FactorDesc &fd,
                                                           const double *__restrict__ poses) {
  double R[9], t[3];
  relative_pose64(poses + 12 * int64_t(fd.pose_i), poses + 12 * int64_t(fd.pose_j), R, t);
  const double s = fd.scale;
  FactorConsts k;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    k.S[i] = float(s * R[i]);
    k.R[i] = float(R[i]);
    k.R64[i] = R[i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    k.u[i] = float(s * t[i]);
    k.t[i] = float(t[i]);
    k.t64[i] = t[i];
  }
  return k;
}

// The same, computed by every lane of a wave (fd is the same in all lanes)
// and held as wave-uniform values.
__device__ __forceinline__ FactorConsts factor_consts(const FactorDesc &fd,
                                                      const double *__restrict__ poses) {
  const FactorConsts l = factor_consts_lane(fd, poses);
  FactorConsts k;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    k.S[i] = uniform_f(l.S[i]);
    k.R[i] = uniform_f(l.R[i]);
    k.R64[i] = uniform_d(l.R64[i]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    k.u[i] = uniform_f(l.u[i]);
    k.t[i] = uniform_f(l.t[i]);
    k.t64[i] = uniform_d(l.t64[i]);
  }
  return k;
}

// Pending hits of one wave, a ring in LDS (structure of arrays).  A lookup
// phase appends the lanes that found their voxel; the math then runs on full
// batches of 64 hits, so misses cost no math lanes.
constexpr int kChunk = kLookupPasses;  // lookup passes per phase of k_linearize (4 waves/SIMD)
constexpr int kOvlChunk = 2;  // lookup passes per step of k_overlap (8 waves/SIMD)
constexpr uint32_t kRing = 64 * kChunk + 64;  // >= 63 left over + 64 * kChunk appended
// Occupancy words of the largest bitset that each thread of a block stages.
constexpr int kOccWordsPerThread = int(kOccMaxBits / 32 / kBlock);
static_assert(kOccWordsPerThread * kBlock * 32 == int(kOccMaxBits), "whole words per thread");

// Start of a tile, in two steps around the caller's work that needs no
// memory: tile_loads loads this thread's share of the map's occupancy words
// and each lane's coordinates of the first NP passes (points threadIdx.x +
// p kBlock of the tile), the words first; tile_stage then stores the words in
// the block's LDS.  The wait for the words leaves the coordinates in flight
// across the caller's barrier.  Words past the bitset and points past the
// tile read zeros without a memory request.  (A block that runs several tiles
// of one map stores the same words again.)
template <int NP>
__device__ __forceinline__ void tile_loads(const FactorDesc &fd, const CloudRsrc &cx,
                                           uint32_t ow[kOccWordsPerThread], float cur[NP][3]) {
  const Rsrc ro = make_rsrc(fd.occ, 4ull * ((fd.occ_mask + 1u) >> 5));
#pragma unroll
  for (int j = 0; j < kOccWordsPerThread; ++j)
    ow[j] = __builtin_bit_cast(uint32_t, ld_f32(ro, (threadIdx.x + uint32_t(j) * kBlock) * 4u));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int p = 0; p < NP; ++p) load_xyz(cx, threadIdx.x + uint32_t(p) * kBlock, cur[p]);
  __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void tile_stage(const FactorDesc &fd, uint32_t *occ_lds,
                                           const uint32_t ow[kOccWordsPerThread]) {
  const uint32_t words = (fd.occ_mask + 1u) >> 5;
#pragma unroll
  for (int j = 0; j < kOccWordsPerThread; ++j) {
    const uint32_t w = threadIdx.x + uint32_t(j) * kBlock;
    if (w < words) occ_lds[w] = ow[j];
  }
}

struct HitQueue {
  float x[kRing], y[kRing], z[kRing];
  int32_t idx[kRing];   // point index in the tile
  int32_t pidx[kRing];  // index of its voxel in the target map's dense arrays
};

static_assert(64 * Sums<VGICP_ACC_MIXED, kNumSums>::kStride * sizeof(float) <= sizeof(HitQueue),
              "the transposed wave sums fit a wave's hit ring");
static_assert(64 * Sums<VGICP_ACC_F32_COMP, kNumSums>::kStride * sizeof(float) <= sizeof(HitQueue),
              "the transposed wave sums fit a wave's hit ring");

__device__ __forceinline__ uint32_t ring_add(uint32_t e, uint32_t d) {
  e += d;  // e < kRing and d < kRing, so one wrap suffices
  if constexpr ((kRing & (kRing - 1)) == 0) return e & (kRing - 1);
  return e >= kRing ? e - kRing : e;
}

// One batch of hits held in registers between its loads and its math.
struct Batch {
  float x, y, z;
  int32_t idx;
  float c[6];    // point covariance
  f32x4 w0, w1;  // voxel statistics: mean (w0.xyz), cov xx..yz (w0.w, w1)
  float czz;     // voxel statistics: cov zz
  int32_t ord;   // voxel ordinal (loaded only for the corr output)
};

// Reads the entry of each lane and issues its buffer loads (no branches:
// dead lanes of a partial batch read entry `head`, point 0 and voxel 0).  Only
// words that are used are loaded: a dead destination register could be
// reused while its load is in flight, which forces an early wait.
template <bool CORR>
__device__ __forceinline__ void batch_load(Batch &B, const HitQueue &Q, uint32_t e, bool live,
                                           Rsrc rc, Rsrc rs, Rsrc ri) {
  B.x = Q.x[e];
  B.y = Q.y[e];
  B.z = Q.z[e];
  const int32_t idx = Q.idx[e];
  const int32_t pidx = Q.pidx[e];
  B.idx = live ? idx : 0;
  // the point's covariance: 24 contiguous bytes, two 12-byte loads (the
  // index is within the tile, below 2^20: a 24-bit multiply)
  const uint32_t co = (uint32_t(B.idx) & 0xffffffu) * 24u;
  const f32x3 c0 = ld_f32x3<kNT>(rc, co), c1 = ld_f32x3<kNT>(rc, co + 12u);
  B.c[0] = c0.x, B.c[1] = c0.y, B.c[2] = c0.z;
  B.c[3] = c1.x, B.c[4] = c1.y, B.c[5] = c1.z;
  // the voxel's statistics: 36 packed bytes
  const uint32_t v = uint32_t(live ? pidx : 0);
  const uint32_t so = v * 36u;
  B.w0 = ld_f32x4(rs, so);
  B.w1 = ld_f32x4(rs, so + 16u);
  B.czz = ld_f32(rs, so + 32u);
  if constexpr (CORR) B.ord = __builtin_bit_cast(int32_t, ld_f32(ri, (v << 4) + 8u));
  // keep the other batch's math below these loads (hoisting it would make it
  // wait for that batch's loads before these are issued)
  __builtin_amdgcn_sched_barrier(0);
}

// Per-point correspondence output of one tile: the value of the tile's point
// `local` goes to the caller's index of that point (through the factor's
// permutation when its source is a reordered copy).
struct CorrOut {
  int32_t *base;        // corr + corr_offset (+ tile begin without a permutation)
  const int32_t *perm;  // permutation from the tile's first point, or NULL
  __device__ __forceinline__ void put(uint32_t local, int32_t v) const {
    base[perm ? uint32_t(perm[local]) : local] = v;
  }
};

template <bool CORR>
__device__ __forceinline__ CorrOut corr_out(int32_t *corr, const FactorDesc &fd, uint32_t begin) {
  if constexpr (!CORR) return {nullptr, nullptr};
  if (fd.perm) return {corr + fd.corr_offset, fd.perm + begin};
  return {corr + fd.corr_offset + begin, nullptr};
}

template <bool LIN, bool R64, bool CORR, int FUSE, bool PAIR, typename SumsT>
__device__ __forceinline__ void batch_math(SumsT &acc, const Batch &B, const FactorConsts &k,
                                           float kappa, const CorrOut &pcorr, uint32_t &nwide,
                                           uint32_t &ndeg) {
  if constexpr (CORR) pcorr.put(uint32_t(B.idx), B.ord);
  const float m[3] = {B.w0.x, B.w0.y, B.w0.z};
  const float S[6] = {B.w0.w, B.w1.x, B.w1.y, B.w1.z, B.w1.w, B.czz};
  if constexpr (PAIR) {
    float e[3], q[3];
    if constexpr (R64) {
      residual64_target(k.R64, k.t64, B.x, B.y, B.z, m, e, q);
    } else {
#pragma clang fp contract(off)
      transform_fp32(k.R, k.t, B.x, B.y, B.z, q);
      e[0] = m[0] - q[0], e[1] = m[1] - q[1], e[2] = m[2] - q[2];
    }
    const bool ok = add_pair_terms<FUSE>(acc, k, kappa, B.x, B.y, B.z, B.c, e, q, S, nwide);
    ndeg += uint32_t(__popcll(__ballot(!ok)));
    return;
  }
  float r[3];
  if constexpr (R64) {
    residual64(k.R64, k.t64, B.x, B.y, B.z, m, r);
  } else {
#pragma clang fp contract(off)
    // e = m - T mu in FP32 (target frame), then rotated into the source frame
    float q[3];
    transform_fp32(k.R, k.t, B.x, B.y, B.z, q);
    const float e0 = m[0] - q[0], e1 = m[1] - q[1], e2 = m[2] - q[2];
    const float *R = k.R;
    r[0] = __builtin_fmaf(R[6], e2, __builtin_fmaf(R[3], e1, R[0] * e0));
    r[1] = __builtin_fmaf(R[7], e2, __builtin_fmaf(R[4], e1, R[1] * e0));
    r[2] = __builtin_fmaf(R[8], e2, __builtin_fmaf(R[5], e1, R[2] * e0));
  }
  const bool ok = add_correspondence<LIN, FUSE>(acc, k, kappa, B.x, B.y, B.z, B.c, r, S, nwide);
  // hits of this batch whose fused covariance was degenerate (wave-uniform)
  ndeg += uint32_t(__popcll(__ballot(!ok)));
}

// Linearization (LIN) or cost evaluation (!LIN) of one tile by one block.
// R64: residual in FP64 from the FP64 relative pose (else plain FP32).
// CORR: also write each point's voxel ordinal (or -1).
// FUSE: how each hit's fused information is formed (kFuse64, kFuse32,
// kFuseGate; see add_correspondence).
//
// Each wave alternates two phases over its 64-point columns of the tile:
//   lookup: kChunk passes of transform + key, one key load and the prefetch
//           of the next pass's coordinates (a fixed set of loads per pass, so
//           the key wait never waits for the prefetch); hits are appended to
//           the wave's ring;
//   math:   the full batches of 64 hits, double-buffered: a batch's voxel
//           and covariance gathers are in flight during the previous batch's
//           math.
// The last partial batch runs at the end of the tile.  FP32 and compensated
// accumulation ask for 4 waves per SIMD (at most 128 VGPRs; both keep one
// FP32 sum per lane); the FP64 accumulators hold twice the registers and
// keep them.
template <int ACC, int N>
struct LinearizeLds {
  typename Sums<ACC, N>::lds_t sums[kWaves * N];
  int cnt[kWaves];
  int wide[kWaves];
  int deg[kWaves];
  HitQueue queues[kWaves];
  uint32_t occ[kOccMaxBits / 32];
  uint8_t up[kUpTable];
};

// Sums per lane of one tile of k_linearize.
template <bool LIN, bool PAIR>
constexpr int tile_sums() {
  return PAIR ? kNumPairSums : LIN ? kNumSums : 1;
}

// PAIR: the pair form's 91 sums of the tile go to partials_pair (stride
// kPairStride), its counters to partials as in the source-frame form.
template <int ACC, bool LIN, bool R64, bool CORR, int FUSE, bool PAIR = false>
__device__ __forceinline__ void linearize_tile(
    LinearizeLds<ACC, tile_sums<LIN, PAIR>()> &L, int64_t tile,
    const FactorDesc *__restrict__ factors, const Tile *__restrict__ tiles,
    const double *__restrict__ poses, const FactorConsts *__restrict__ consts,
    double *__restrict__ partials, int32_t *__restrict__ corr, float kappa,
    double *__restrict__ partials_pair = nullptr) {
  static_assert(!PAIR || (LIN && !CORR), "the pair form linearizes without correspondences");
  constexpr int N = tile_sums<LIN, PAIR>();
  using SumsT = Sums<ACC, N>;
  auto &lds = L.sums;
  auto &lds_cnt = L.cnt;
  auto &lds_wide = L.wide;
  auto &lds_deg = L.deg;
  auto &queues = L.queues;
  uint32_t *occ_lds = L.occ;

  const Tile td = tiles[tile];
  if (td.factor < 0) return;  // padding (uniform over the block)
  const FactorDesc fd = factors[td.factor];
  const uint32_t n = uint32_t(fd.n);
  const uint32_t begin = uint32_t(td.start);
  const uint32_t end = min(begin + uint32_t(fd.tile_points), n);
  const CloudRsrc cx = tile_rsrc(fd.xyz, begin, end);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x >> 6;

  // Coordinates of the chunk's kChunk passes (prefetched one chunk ahead;
  // past the tile's end the loads return zeros and the lanes are invalid).
  float cur[kChunk][3];
  uint32_t base = begin + wave * 64;
  uint32_t ow[kOccWordsPerThread];
  tile_loads<kChunk>(fd, cx, ow, cur);
  // the relative pose (from the round's table when there is one) while the
  // loads are in flight.  The gated variant always computes it: compiled with
  // the table's branch it ran 13 % slower on the full-size precision workload.
  FactorConsts k;
  if constexpr (FUSE == kFuseGate)
    k = factor_consts(fd, poses);
  else
    k = consts ? consts[td.factor] : factor_consts(fd, poses);
  // the previous tile's reads of the LDS sums and bits end before this barrier
  tile_stage(fd, occ_lds, ow);
  __syncthreads();
  const Rsrc rc = make_rsrc(fd.cov + 6ull * begin, 24ull * (end - begin));
  const Rsrc rb = make_rsrc(fd.bricks, 32ull << fd.log2cap);
  const Rsrc rs = make_rsrc(fd.stats, 36ull * fd.n_voxels);
  const Rsrc ri = make_rsrc(fd.info, 16ull * fd.n_voxels);
  const CorrOut pcorr = corr_out<CORR>(corr, fd, begin);
  HitQueue &Q = queues[wave];

  SumsT acc;
  acc.zero();
  uint32_t head = 0, count = 0;  // wave-uniform ring state
  uint32_t hits = 0;             // wave-uniform hit count
  uint32_t nwide = 0;            // per lane: hits with the FP64 fused covariance
  uint32_t ndeg = 0;  // hits with a degenerate fused covariance (complete in lane 0)

  while (base < end) {
    // ---- lookup phase: the brick records of all kChunk passes are in flight
    // at once, then the next chunk's coordinates; records are then resolved
    // in order, so each wait leaves the later records and the whole prefetch
    // in flight.
    VoxelKey vk[kChunk];
    RecordLoad rec[kChunk];
    bool occ[kChunk];
#pragma unroll
    for (int p = 0; p < kChunk; ++p) {
      float v[3];
      lookup_coords(k.S, k.u, cur[p][0], cur[p][1], cur[p][2], v);
      vk[p] = voxel_key<true>(v, fd.log2cap, L.up);
      occ[p] = home_occupied(occ_lds, occ_word_mask(fd.occ_mask), vk[p].h);
    }
#pragma unroll
    for (int p = 0; p < kChunk; ++p) rec[p] = load_home(rb, vk[p].h, occ[p]);
    __builtin_amdgcn_sched_barrier(0);
    float nxt[kChunk][3];
#pragma unroll
    for (int p = 0; p < kChunk; ++p)
      load_xyz(cx, base - begin + (kChunk + p) * kBlock + lane, nxt[p]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < kChunk; ++p) {
      const uint32_t i = base + p * kBlock + lane;
      const int h = find_voxel(rb, fd.log2cap, vk[p], rec[p], occ[p]);
      const bool hit = h >= 0 && i < end;
      if constexpr (CORR) {
        if (i < end && !hit) pcorr.put(i - begin, -1);
      }
      const uint64_t mask = __builtin_amdgcn_ballot_w64(hit);
      if (hit) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
            uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
        const uint32_t e = ring_add(ring_add(head, count), below);
        Q.x[e] = cur[p][0];
        Q.y[e] = cur[p][1];
        Q.z[e] = cur[p][2];
        Q.idx[e] = int32_t(i - begin);
        Q.pidx[e] = h;
      }
      const uint32_t got = uint32_t(__popcll(mask));
      count += got;
      hits += got;
    }
#pragma unroll
    for (int p = 0; p < kChunk; ++p)
#pragma unroll
      for (int a = 0; a < 3; ++a) cur[p][a] = nxt[p][a];
    base += kChunk * kBlock;
    __builtin_amdgcn_wave_barrier();
    // ---- math phase: full batches, double-buffered
    const uint32_t nb = count / 64;
    if (nb > 0) {
      // unrolled by two so that the buffers swap roles without copies (a
      // copy would wait for the loads it copies)
      Batch A, B;
      batch_load<CORR>(A, Q, ring_add(head, lane), true, rc, rs, ri);
      head = ring_add(head, 64);
      uint32_t bi = 1;
      for (; bi + 1 < nb; bi += 2) {
        batch_load<CORR>(B, Q, ring_add(head, lane), true, rc, rs, ri);
        head = ring_add(head, 64);
        batch_math<LIN, R64, CORR, FUSE, PAIR>(acc, A, k, kappa, pcorr, nwide, ndeg);
        batch_load<CORR>(A, Q, ring_add(head, lane), true, rc, rs, ri);
        head = ring_add(head, 64);
        batch_math<LIN, R64, CORR, FUSE, PAIR>(acc, B, k, kappa, pcorr, nwide, ndeg);
      }
      if (bi < nb) {
        batch_load<CORR>(B, Q, ring_add(head, lane), true, rc, rs, ri);
        head = ring_add(head, 64);
        batch_math<LIN, R64, CORR, FUSE, PAIR>(acc, A, k, kappa, pcorr, nwide, ndeg);
        batch_math<LIN, R64, CORR, FUSE, PAIR>(acc, B, k, kappa, pcorr, nwide, ndeg);
      } else {
        batch_math<LIN, R64, CORR, FUSE, PAIR>(acc, A, k, kappa, pcorr, nwide, ndeg);
      }
      count -= nb * 64;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (count > 0) {  // last partial batch: dead lanes add nothing
    const bool live = lane < count;
    Batch A;
    batch_load<CORR>(A, Q, ring_add(head, live ? lane : 0), live, rc, rs, ri);
    if (live) batch_math<LIN, R64, CORR, FUSE, PAIR>(acc, A, k, kappa, pcorr, nwide, ndeg);
  }

  // the ring is empty: its LDS holds the transposed sums now
  acc.reduce_to(lds, wave, lane, reinterpret_cast<float *>(&Q));
  // hits that formed F' in FP64: counted with the gate, all hits with kFuse64
  const int wide = FUSE == kFuseGate ? wave_sum(int(nwide)) : FUSE == kFuse64 ? int(hits) : 0;
  if (lane == kLastLane) {
    lds_cnt[wave] = int(hits);
    lds_wide[wave] = wide;
  }
  // lane 0 took part in every batch (the last, partial one included)
  if (lane == 0) lds_deg[wave] = int(ndeg);
  __syncthreads();
  double *__restrict__ out = partials + tile * kPartialStride;
  static_assert(N <= kBlock - 3, "the counters' threads hold no sum");
  if (threadIdx.x < N) {
    const double v = SumsT::finish(lds, threadIdx.x);
    if constexpr (PAIR)
      partials_pair[tile * kPairStride + threadIdx.x] = v;
    else
      out[LIN ? threadIdx.x : 27] = v;
  } else if (threadIdx.x == kBlock - 3) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += lds_cnt[w];
    out[kNumSums] = double(s);
  } else if (threadIdx.x == kBlock - 2) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += lds_wide[w];
    out[kWideSlot] = double(s);
  } else if (threadIdx.x == kBlock - 1) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += lds_deg[w];
    out[kDegenerateSlot] = double(s);
  }
}

// Linearization (LIN) or cost evaluation (!LIN) of the tiles [tile_base,
// tile_end).  The grid is a multiple of 8; XCD x (blocks are dealt round-robin
// over the 8 XCDs) takes the x-th eighth of the tile range, and its P blocks
// walk it in order (block l: tiles l, l + P, l + 2P, ... of the range), so the
// tiles in flight on one XCD are neighbours in the table: tiles of one factor,
// and factors sorted by target map, share that XCD's L2.  With one block per
// tile (P = the eighth's length) each block runs one tile; a persistent grid
// (P blocks per XCD resident at once) runs several.  Every tile stages its
// map's occupancy bits in the block's LDS.
template <int ACC, bool LIN, bool R64, bool CORR, int FUSE>
__global__ void __launch_bounds__(kBlock, ACC == VGICP_ACC_F64 ? 1 : 4)
k_linearize(const FactorDesc *__restrict__ factors, const Tile *__restrict__ tiles,
            int64_t tile_base, int64_t tile_end, int32_t tile_stride,
            const double *__restrict__ poses, const FactorConsts *__restrict__ consts,
            double *__restrict__ partials, int32_t *__restrict__ corr, float kappa) {
  __shared__ LinearizeLds<ACC, LIN ? kNumSums : 1> L;
  // tile indices are below 2^31 (the tile table is indexed by int32)
  const uint32_t base = uint32_t(tile_base), count = uint32_t(tile_end - tile_base);
  const uint32_t per = (count + 7u) >> 3;
  const uint32_t lo = (blockIdx.x & 7u) * per;
  const uint32_t hi = min(lo + per, count);
  const uint32_t P = gridDim.x >> 3;
  up_table_fill(L.up);  // read after the first tile's barrier
  for (uint32_t t = lo + (blockIdx.x >> 3); t < hi; t += P)
    linearize_tile<ACC, LIN, R64, CORR, FUSE>(L, int64_t(base) + int64_t(t) * tile_stride,
                                              factors, tiles, poses, consts, partials, corr,
                                              kappa);
}

// The pair form (Eqs. (5)-(6) term by term) over the tiles [tile_base,
// tile_end), tiles dealt as in k_linearize.  Its 91 FP32 sums per lane take
// about 200 VGPRs: 2 waves per SIMD.
template <int ACC, bool R64, int FUSE>
__global__ void __launch_bounds__(kBlock, 2)
k_linearize_pair(const FactorDesc *__restrict__ factors, const Tile *__restrict__ tiles,
                 int64_t tile_base, int64_t tile_end, int32_t tile_stride,
                 const double *__restrict__ poses, const FactorConsts *__restrict__ consts,
                 double *__restrict__ partials, double *__restrict__ partials_pair,
                 float kappa) {
  __shared__ LinearizeLds<ACC, kNumPairSums> L;
  const uint32_t base = uint32_t(tile_base), count = uint32_t(tile_end - tile_base);
  const uint32_t per = (count + 7u) >> 3;
  const uint32_t lo = (blockIdx.x & 7u) * per;
  const uint32_t hi = min(lo + per, count);
  const uint32_t P = gridDim.x >> 3;
  up_table_fill(L.up);  // read after the first tile's barrier
  for (uint32_t t = lo + (blockIdx.x >> 3); t < hi; t += P)
    linearize_tile<ACC, true, R64, false, FUSE, true>(
        L, int64_t(base) + int64_t(t) * tile_stride, factors, tiles, poses, consts, partials,
        nullptr, kappa, partials_pair);
}

// Overlap hit count of one tile (Eq. (7)): brick records only.
__device__ __forceinline__ void overlap_tile(int *lds_cnt, uint32_t *occ_lds,
                                             const uint8_t *up_lds, int64_t tile,
                                             const FactorDesc *__restrict__ factors,
                                             const Tile *__restrict__ tiles,
                                             const double *__restrict__ poses,
                                             double *__restrict__ partials) {
  const Tile td = tiles[tile];
  if (td.factor < 0) return;  // padding (uniform over the block)
  const FactorDesc fd = factors[td.factor];
  const uint32_t n = uint32_t(fd.n);
  const uint32_t begin = uint32_t(td.start);
  const uint32_t end = min(begin + uint32_t(fd.tile_points), n);
  const CloudRsrc cx = tile_rsrc(fd.xyz, begin, end);
  float cur[kOvlChunk][3];
  uint32_t base = begin + (threadIdx.x & ~63u);
  const uint32_t lane = threadIdx.x & 63;
  uint32_t ow[kOccWordsPerThread];
  tile_loads<kOvlChunk>(fd, cx, ow, cur);
  // the relative pose while the loads are in flight
  const FactorConsts k = factor_consts(fd, poses);
  // the previous tile's reads of the LDS counts and bits end before this barrier
  tile_stage(fd, occ_lds, ow);
  __syncthreads();
  const Rsrc rb = make_rsrc(fd.bricks, 32ull << fd.log2cap);
  int hits = 0;
  for (; base < end; base += kOvlChunk * kBlock) {
    VoxelKey vk[kOvlChunk];
    RecordLoad rec[kOvlChunk];
    bool occ[kOvlChunk];
#pragma unroll
    for (int p = 0; p < kOvlChunk; ++p) {
      float v[3];
      lookup_coords(k.S, k.u, cur[p][0], cur[p][1], cur[p][2], v);
      vk[p] = voxel_key<true>(v, fd.log2cap, up_lds);
      occ[p] = home_occupied(occ_lds, occ_word_mask(fd.occ_mask), vk[p].h);
    }
#pragma unroll
    for (int p = 0; p < kOvlChunk; ++p) rec[p] = load_home(rb, vk[p].h, occ[p]);
    __builtin_amdgcn_sched_barrier(0);
    float nxt[kOvlChunk][3];
#pragma unroll
    for (int p = 0; p < kOvlChunk; ++p)
      load_xyz(cx, base - begin + (kOvlChunk + p) * kBlock + lane, nxt[p]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < kOvlChunk; ++p) {
      const bool valid = base + p * kBlock + lane < end;
      const int hs = find_voxel(rb, fd.log2cap, vk[p], rec[p], occ[p]);
      hits += (valid && hs >= 0) ? 1 : 0;
    }
#pragma unroll
    for (int p = 0; p < kOvlChunk; ++p)
#pragma unroll
      for (int a = 0; a < 3; ++a) cur[p][a] = nxt[p][a];
  }
  hits = wave_sum(hits);
  if ((threadIdx.x & 63) == kLastLane) lds_cnt[threadIdx.x >> 6] = hits;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += lds_cnt[w];
    partials[tile * kPartialStride + kNumSums] = double(s);
  }
}

// Overlap hit counts of the tiles [tile_base, tile_end), tiles dealt to
// blocks as in k_linearize.
__global__ void __launch_bounds__(kBlock)
k_overlap(const FactorDesc *__restrict__ factors, const Tile *__restrict__ tiles,
          int64_t tile_base, int64_t tile_end, int32_t tile_stride,
          const double *__restrict__ poses, double *__restrict__ partials) {
  __shared__ int lds_cnt[kWaves];
  __shared__ uint32_t occ_lds[kOccMaxBits / 32];
  __shared__ uint8_t up_lds[kUpTable];
  const uint32_t base = uint32_t(tile_base), count = uint32_t(tile_end - tile_base);
  const uint32_t per = (count + 7u) >> 3;
  const uint32_t lo = (blockIdx.x & 7u) * per;
  const uint32_t hi = min(lo + per, count);
  const uint32_t P = gridDim.x >> 3;
  up_table_fill(up_lds);  // read after the first tile's barrier
  for (uint32_t t = lo + (blockIdx.x >> 3); t < hi; t += P)
    overlap_tile(lds_cnt, occ_lds, up_lds, int64_t(base) + int64_t(t) * tile_stride,
                 factors, tiles, poses, partials);
}

// ---------------------------------------------------------------- target order
// Sort keys for putting each factor's source points in the order of the
// target voxels they fall in at the given poses: for point i of factor f (in
// the factor set's current copy), the index of its voxel in the map's dense
// arrays (brick after brick, Morton order within a brick: the order of the
// statistics records a round reads) or 0xffffffff for a point in no voxel,
// with f in the high 32 bits; the value is i.  Keys go to the factor's
// per-point output range (corr_offset).  One 256-thread block per tile,
// blocks in tile order.
__global__ void __launch_bounds__(kBlock)
k_voxel_order_keys(const FactorDesc *__restrict__ factors, const Tile *__restrict__ tiles,
                   int64_t n_tiles, const double *__restrict__ poses,
                   uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const Tile td = tiles[tile];
  if (td.factor < 0) return;  // padding
  const FactorDesc fd = factors[td.factor];
  const FactorConsts k = factor_consts(fd, poses);
  const uint32_t n = uint32_t(fd.n);
  const uint32_t begin = uint32_t(td.start);
  const uint32_t end = min(begin + uint32_t(fd.tile_points), n);
  const CloudRsrc cx = tile_rsrc(fd.xyz, begin, end);
  const Rsrc rb = make_rsrc(fd.bricks, 32ull << fd.log2cap);
  const uint64_t hi = uint64_t(uint32_t(td.factor)) << 32;
  // whole waves run every pass (the ballot in find_voxel); lanes past the
  // tile's end read zeros and write nothing
  for (uint32_t i0 = begin; i0 < end; i0 += kBlock) {
    const uint32_t i = i0 + threadIdx.x;
    float p[3];
    load_xyz(cx, i - begin, p);
    float v[3];
    lookup_coords(k.S, k.u, p[0], p[1], p[2], v);
    const VoxelKey vk = voxel_key(v, fd.log2cap);
    const RecordLoad rec = load_home(rb, vk.h, true);
    const int h = find_voxel(rb, fd.log2cap, vk, rec, true);
    if (i < end) {
      keys[fd.corr_offset + i] = hi | (h >= 0 ? uint64_t(uint32_t(h)) : 0xffffffffull);
      vals[fd.corr_offset + i] = i;
    }
  }
}

hipError_t launch_voxel_order_keys(const vgicp_factorset_s *fs, const double *poses,
                                   uint64_t *keys, uint32_t *vals, hipStream_t st) {
  if (fs->n_tiles <= 0) return hipSuccess;
  k_voxel_order_keys<<<unsigned(fs->n_tiles), kBlock, 0, st>>>(
      fs->d_factors, fs->d_tiles, fs->n_tiles, poses, keys, vals);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reduce
// One 64-lane block per factor: add the factor's tile partials in tile order
// (FP64), then expand the source-frame system to the 12x12 Hessian factor.
//   mode 0: linearize (H, b, e, inliers)   1: cost only (e, inliers)
//   mode 2: overlap (hits, overlap)
__global__ void __launch_bounds__(64)
k_reduce(const FactorDesc *__restrict__ factors, int64_t factor_base,
         const double *__restrict__ poses, const double *__restrict__ partials, int mode,
         double *__restrict__ H, double *__restrict__ b, double *__restrict__ e,
         int64_t *__restrict__ inl, double *__restrict__ overlap) {
  __shared__ double s[kPartialStride];
  __shared__ double Hr[36], Ad[36], K[36], Hjj[36];
  const int64_t f = factor_base + blockIdx.x;
  const FactorDesc fd = factors[f];
  const int lane = threadIdx.x;
  if (lane <= kNumSums) {
    double acc = 0.0;
    const bool used = (mode == 0) || lane >= 27;
    if (used)
      for (int32_t tt = 0; tt < fd.n_tiles; ++tt)
        acc += partials[(fd.tile_begin + int64_t(tt) * fd.tile_stride) * kPartialStride + lane];
    s[lane] = acc;
  }
  __syncthreads();
  if (mode == 2) {
    if (lane == 0) {
      const int64_t hits = int64_t(s[kNumSums]);
      inl[f] = hits;
      if (overlap) overlap[f] = fd.n > 0 ? double(hits) / double(fd.n) : 0.0;
    }
    return;
  }
  if (lane == 0) {
    e[f] = s[27];
    inl[f] = int64_t(s[kNumSums]);
  }
  if (mode == 1) return;

  // source-frame 6x6 from its upper triangle
  if (lane < 36) {
    const int r = lane / 6, c = lane % 6;
    const int lo = r < c ? r : c, hi = r < c ? c : r;
    // index of (lo, hi) in the row-major upper triangle
    const int idx = lo * 6 - lo * (lo - 1) / 2 + (hi - lo);
    Hr[lane] = s[idx];
  }
  if (lane == 0) {
    double R[9], t[3];
    relative_pose64(poses + 12 * int64_t(fd.pose_i), poses + 12 * int64_t(fd.pose_j), R, t);
    // Ad(T^-1) = [[R^T, 0], [-R^T [t]x, R^T]] in (omega, rho) order
    const double tx[9] = {0.0, -t[2], t[1], t[2], 0.0, -t[0], -t[1], t[0], 0.0};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const double RT = R[3 * c + r];
        double RTt = 0.0;
        for (int a = 0; a < 3; ++a) RTt += R[3 * a + r] * tx[3 * a + c];
        Ad[6 * r + c] = RT;
        Ad[6 * r + 3 + c] = 0.0;
        Ad[6 * (3 + r) + c] = -RTt;
        Ad[6 * (3 + r) + 3 + c] = RT;
      }
  }
  __syncthreads();
  if (lane < 36) {  // K = Hr Ad
    const int r = lane / 6, c = lane % 6;
    double a = 0.0;
    for (int k = 0; k < 6; ++k) a += Hr[6 * r + k] * Ad[6 * k + c];
    K[lane] = a;
  }
  __syncthreads();
  if (lane < 36) {  // Hjj = Ad^T K, upper triangle mirrored
    const int r = lane / 6, c = lane % 6;
    const int lo = r < c ? r : c, hi = r < c ? c : r;
    double a = 0.0;
    for (int k = 0; k < 6; ++k) a += Ad[6 * k + lo] * K[6 * k + hi];
    Hjj[lane] = a;
  }
  __syncthreads();
  double *__restrict__ Hf = H + f * 144;
  for (int idx = lane; idx < 144; idx += 64) {
    const int r = idx / 12, c = idx % 12;
    double v;
    if (r < 6 && c < 6) v = Hr[6 * r + c];
    else if (r < 6) v = -K[6 * r + (c - 6)];            // H_ij
    else if (c < 6) v = -K[6 * c + (r - 6)];            // H_ij^T
    else v = Hjj[6 * (r - 6) + (c - 6)];
    Hf[idx] = v;
  }
  if (lane < 6) {
    b[f * 12 + lane] = s[21 + lane];
  } else if (lane < 12) {
    const int c = lane - 6;
    double a = 0.0;
    for (int k = 0; k < 6; ++k) a += Ad[6 * k + c] * s[21 + k];
    b[f * 12 + lane] = -a;
  }
}

// Pair form: one 64-lane block per factor adds the factor's tile partials in
// tile order (FP64) and writes the 12 x 12 H from its upper triangle, b, e
// and the inliers.
__global__ void __launch_bounds__(64)
k_reduce_pair(const FactorDesc *__restrict__ factors, int64_t factor_base,
              const double *__restrict__ partials, const double *__restrict__ partials_pair,
              double *__restrict__ H, double *__restrict__ b, double *__restrict__ e,
              int64_t *__restrict__ inl) {
  __shared__ double s[kPairStride];
  const int64_t f = factor_base + blockIdx.x;
  const FactorDesc fd = factors[f];
  const int lane = threadIdx.x;
  for (int i = lane; i < kNumPairSums; i += 64) {
    double acc = 0.0;
    for (int32_t tt = 0; tt < fd.n_tiles; ++tt)
      acc += partials_pair[(fd.tile_begin + int64_t(tt) * fd.tile_stride) * kPairStride + i];
    s[i] = acc;
  }
  if (lane == 0) {
    double hits = 0.0;
    for (int32_t tt = 0; tt < fd.n_tiles; ++tt)
      hits += partials[(fd.tile_begin + int64_t(tt) * fd.tile_stride) * kPartialStride + kNumSums];
    inl[f] = int64_t(hits);
  }
  __syncthreads();
  double *__restrict__ Hf = H + f * 144;
  for (int idx = lane; idx < 144; idx += 64) {
    const int r = idx / 12, c = idx % 12;
    Hf[idx] = r <= c ? s[pair_index(r, c)] : s[pair_index(c, r)];
  }
  if (lane < 12) b[f * 12 + lane] = s[78 + lane];
  if (lane == 0) e[f] = s[90];
}

// ---------------------------------------------------------------- assembly
// One 64-lane block per pose: lanes 0..35 own an entry of the 6x6 diagonal
// block, lanes 36..41 an entry of b.  Contributions are added in CSR order
// (factor order), so the sums are deterministic.  An entry is factor * 4 +
// side (0: the pose is the factor's pose i, 1: pose j) + 2 when the factor's
// two poses coincide; such a factor's pose-i entry also adds H_ij + H_ij^T.
__global__ void __launch_bounds__(64)
k_assemble_diag(const int64_t *__restrict__ off, const int64_t *__restrict__ ent,
                const double *__restrict__ H, const double *__restrict__ b,
                double *__restrict__ Hdiag, double *__restrict__ bvec) {
  const int p = blockIdx.x, lane = threadIdx.x;
  if (lane >= 42) return;
  double acc = 0.0;
  for (int64_t k = off[p]; k < off[p + 1]; ++k) {
    const int64_t f = ent[k] >> 2;
    const int o = 6 * (ent[k] & 1);
    if (lane < 36) {
      const int r = lane / 6, c = lane % 6;
      acc += H[f * 144 + (o + r) * 12 + (o + c)];
      if (ent[k] & 2) acc += H[f * 144 + r * 12 + (6 + c)] + H[f * 144 + (6 + r) * 12 + c];
    } else {
      acc += b[f * 12 + o + (lane - 36)];
    }
  }
  if (lane < 36)
    Hdiag[int64_t(p) * 36 + lane] = acc;
  else
    bvec[int64_t(p) * 6 + (lane - 36)] = acc;
}

// One 64-lane block per unordered pose pair (p, q), p < q: block (p, q) is the
// sum of H_ij over factors (i, j) = (p, q) and of H_ij^T over (i, j) = (q, p).
__global__ void __launch_bounds__(64)
k_assemble_pairs(const int64_t *__restrict__ off, const int64_t *__restrict__ ent,
                 const double *__restrict__ H, double *__restrict__ Hoff) {
  const int q = blockIdx.x, lane = threadIdx.x;
  if (lane >= 36) return;
  const int r = lane / 6, c = lane % 6;
  double acc = 0.0;
  for (int64_t k = off[q]; k < off[q + 1]; ++k) {
    const int64_t f = ent[k] >> 1;
    const bool flip = ent[k] & 1;
    acc += flip ? H[f * 144 + (6 + r) * 12 + c] : H[f * 144 + r * 12 + (6 + c)];
  }
  Hoff[int64_t(q) * 36 + lane] = acc;
}

// ---------------------------------------------------------------- launchers
static inline unsigned xcd_grid(int64_t tiles) { return unsigned(((tiles + 7) / 8) * 8); }

// Grid of a launch over `tiles` tiles: one block per tile, or with a
// persistent schedule (persist_blocks > 0) at most persist_blocks blocks
// (a multiple of 8), each walking several tiles.
static inline unsigned tile_grid(int64_t tiles, int32_t persist_blocks) {
  const unsigned one_per_tile = xcd_grid(tiles);
  if (persist_blocks <= 0) return one_per_tile;
  return std::min(one_per_tile, unsigned(persist_blocks));
}

template <int ACC, bool LIN, bool R64, int FUSE>
static hipError_t launch_lin(const vgicp_factorset_s *fs, int64_t tb, int64_t te, int32_t stride,
                             const double *poses, const FactorConsts *consts, double *partials,
                             int32_t *corr, float kappa, hipStream_t st) {
  if (te <= tb) return hipSuccess;
  const unsigned grid = tile_grid(te - tb, fs->persist_blocks);
  if (corr) {
    k_linearize<ACC, LIN, R64, true, FUSE><<<grid, kBlock, 0, st>>>(
        fs->d_factors, fs->d_tiles, tb, te, stride, poses, consts, partials, corr, kappa);
  } else {
    k_linearize<ACC, LIN, R64, false, FUSE><<<grid, kBlock, 0, st>>>(
        fs->d_factors, fs->d_tiles, tb, te, stride, poses, consts, partials, nullptr,
        kappa);
  }
  return hipGetLastError();
}

template <int ACC, int FUSE>
static hipError_t launch_acc(const vgicp_factorset_s *fs, bool lin, bool r64, int64_t tb,
                             int64_t te, int32_t stride, const double *poses,
                             const FactorConsts *consts, double *partials, int32_t *corr,
                             float kappa, hipStream_t st) {
  if (lin) {
    return r64 ? launch_lin<ACC, true, true, FUSE>(fs, tb, te, stride, poses, consts, partials,
                                                   corr, kappa, st)
               : launch_lin<ACC, true, false, FUSE>(fs, tb, te, stride, poses, consts, partials,
                                                    corr, kappa, st);
  }
  return r64 ? launch_lin<ACC, false, true, FUSE>(fs, tb, te, stride, poses, consts, partials,
                                                  corr, kappa, st)
             : launch_lin<ACC, false, false, FUSE>(fs, tb, te, stride, poses, consts, partials,
                                                   corr, kappa, st);
}

template <int FUSE>
static hipError_t launch_k(const vgicp_factorset_s *fs, int accum, bool lin, bool r64, int64_t tb,
                           int64_t te, int32_t stride, const double *poses,
                           const FactorConsts *consts, double *partials, int32_t *corr,
                           float kappa, hipStream_t st) {
  switch (accum) {
    case VGICP_ACC_F64:
      return launch_acc<VGICP_ACC_F64, FUSE>(fs, lin, r64, tb, te, stride, poses, consts,
                                              partials, corr, kappa, st);
    case VGICP_ACC_F32_COMP:
      return launch_acc<VGICP_ACC_F32_COMP, FUSE>(fs, lin, r64, tb, te, stride, poses, consts,
                                                   partials, corr, kappa, st);
    case VGICP_ACC_F32:
      return launch_acc<VGICP_ACC_F32, FUSE>(fs, lin, r64, tb, te, stride, poses, consts,
                                              partials, corr, kappa, st);
    default:
      return launch_acc<VGICP_ACC_MIXED, FUSE>(fs, lin, r64, tb, te, stride, poses, consts,
                                                partials, corr, kappa, st);
  }
}

// Blocks of the linearization kernel for (accum, fused, form) one CU holds at once.
hipError_t linearize_blocks_per_cu(int accum, int fused, int form, int *blocks) {
  const void *fn;
  const bool f64 = fused == VGICP_FUSED_F64;
  if (form == VGICP_FORM_PAIR) {
    switch (accum) {
      case VGICP_ACC_F32_COMP:
        fn = f64 ? (const void *)k_linearize_pair<VGICP_ACC_F32_COMP, true, kFuse64>
                 : (const void *)k_linearize_pair<VGICP_ACC_F32_COMP, true, kFuse32>;
        break;
      case VGICP_ACC_F32:
        fn = f64 ? (const void *)k_linearize_pair<VGICP_ACC_F32, true, kFuse64>
                 : (const void *)k_linearize_pair<VGICP_ACC_F32, true, kFuse32>;
        break;
      default:
        fn = f64 ? (const void *)k_linearize_pair<VGICP_ACC_MIXED, true, kFuse64>
                 : (const void *)k_linearize_pair<VGICP_ACC_MIXED, true, kFuse32>;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, 0);
  }
  switch (accum) {
    case VGICP_ACC_F64:
      fn = f64 ? (const void *)k_linearize<VGICP_ACC_F64, true, true, false, kFuse64>
               : (const void *)k_linearize<VGICP_ACC_F64, true, true, false, kFuse32>;
      break;
    case VGICP_ACC_F32_COMP:
      fn = f64 ? (const void *)k_linearize<VGICP_ACC_F32_COMP, true, true, false, kFuse64>
               : (const void *)k_linearize<VGICP_ACC_F32_COMP, true, true, false, kFuse32>;
      break;
    case VGICP_ACC_F32:
      fn = f64 ? (const void *)k_linearize<VGICP_ACC_F32, true, true, false, kFuse64>
               : (const void *)k_linearize<VGICP_ACC_F32, true, true, false, kFuse32>;
      break;
    default:
      fn = f64 ? (const void *)k_linearize<VGICP_ACC_MIXED, true, true, false, kFuse64>
               : (const void *)k_linearize<VGICP_ACC_MIXED, true, true, false, kFuse32>;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, 0);
}

// Constants of every factor of fs at `poses` into fs->d_consts (one thread
// per factor), for the linearize launches of a round that follow on st.
__global__ void __launch_bounds__(64)
k_factor_consts(const FactorDesc *__restrict__ factors, int64_t n, const double *__restrict__ poses,
                FactorConsts *__restrict__ out) {
  const int64_t f = int64_t(blockIdx.x) * 64 + threadIdx.x;
  if (f >= n) return;
  out[f] = factor_consts_lane(factors[f], poses);
}

hipError_t launch_factor_consts(const vgicp_factorset_s *fs, const double *poses, hipStream_t st) {
  if (!fs->d_consts || fs->n_factors <= 0) return hipSuccess;
  k_factor_consts<<<unsigned((fs->n_factors + 63) / 64), 64, 0, st>>>(
      fs->d_factors, fs->n_factors, poses, static_cast<FactorConsts *>(fs->d_consts));
  return hipGetLastError();
}

// Launches over the tiles tb + k * stride, k < te - tb (stride 1: the range
// [tb, te) of the tile table; a factor's own tiles: its tile_begin, n_tiles
// and tile_stride).  `consts` (may be NULL: every tile computes its factor's
// constants) is the table launch_factor_consts wrote for these poses.
hipError_t launch_linearize_into(const vgicp_factorset_s *fs, int accum, int resid, int fused,
                                 float kappa, bool lin, int64_t tb, int64_t te,
                                 const double *poses, double *partials, int32_t *corr,
                                 hipStream_t st, int32_t stride, const void *consts) {
  const bool r64 = resid == VGICP_RESID_F64;
  const FactorConsts *k = static_cast<const FactorConsts *>(consts);
  if (fused == VGICP_FUSED_F64)
    return launch_k<kFuse64>(fs, accum, lin, r64, tb, te, stride, poses, k, partials, corr, 0.f,
                             st);
  // the gated variant computes the constants in every workgroup (see
  // linearize_tile)
  if (kappa > 0.f)
    return launch_k<kFuseGate>(fs, accum, lin, r64, tb, te, stride, poses, nullptr, partials,
                               corr, kappa, st);
  return launch_k<kFuse32>(fs, accum, lin, r64, tb, te, stride, poses, k, partials, corr, 0.f, st);
}

hipError_t launch_linearize(const vgicp_factorset_s *fs, int accum, int resid, int fused,
                            float kappa, bool lin, int64_t tb, int64_t te, const double *poses,
                            int32_t *corr, hipStream_t st, int32_t stride, const void *consts) {
  return launch_linearize_into(fs, accum, resid, fused, kappa, lin, tb, te, poses,
                               fs->d_partials, corr, st, stride, consts);
}

template <int ACC, int FUSE>
static hipError_t launch_pair_acc(const vgicp_factorset_s *fs, bool r64, int64_t tb, int64_t te,
                                  int32_t stride, const double *poses,
                                  const FactorConsts *consts, double *partials,
                                  double *partials_pair, float kappa, hipStream_t st) {
  const unsigned grid = tile_grid(te - tb, fs->persist_blocks);
  if (r64)
    k_linearize_pair<ACC, true, FUSE><<<grid, kBlock, 0, st>>>(
        fs->d_factors, fs->d_tiles, tb, te, stride, poses, consts, partials,
        partials_pair, kappa);
  else
    k_linearize_pair<ACC, false, FUSE><<<grid, kBlock, 0, st>>>(
        fs->d_factors, fs->d_tiles, tb, te, stride, poses, consts, partials,
        partials_pair, kappa);
  return hipGetLastError();
}

template <int FUSE>
static hipError_t launch_pair_k(const vgicp_factorset_s *fs, int accum, bool r64, int64_t tb,
                                int64_t te, int32_t stride, const double *poses,
                                const FactorConsts *consts, double *partials,
                                double *partials_pair, float kappa, hipStream_t st) {
  switch (accum) {
    case VGICP_ACC_F32_COMP:
      return launch_pair_acc<VGICP_ACC_F32_COMP, FUSE>(fs, r64, tb, te, stride, poses, consts,
                                                        partials, partials_pair, kappa, st);
    case VGICP_ACC_F32:
      return launch_pair_acc<VGICP_ACC_F32, FUSE>(fs, r64, tb, te, stride, poses, consts,
                                                   partials, partials_pair, kappa, st);
    default:
      return launch_pair_acc<VGICP_ACC_MIXED, FUSE>(fs, r64, tb, te, stride, poses, consts,
                                                     partials, partials_pair, kappa, st);
  }
}

hipError_t launch_linearize_pair(const vgicp_factorset_s *fs, int accum, int resid, int fused,
                                 float kappa, int64_t tb, int64_t te, const double *poses,
                                 hipStream_t st, int32_t stride, const void *consts) {
  if (te <= tb) return hipSuccess;
  if (accum == VGICP_ACC_F64) return hipErrorInvalidValue;  // rejected by the callers
  const bool r64 = resid == VGICP_RESID_F64;
  const FactorConsts *k = static_cast<const FactorConsts *>(consts);
  double *pp = fs->d_partials_pair;
  double *part = fs->d_partials;
  if (fused == VGICP_FUSED_F64)
    return launch_pair_k<kFuse64>(fs, accum, r64, tb, te, stride, poses, k, part, pp, 0.f, st);
  if (kappa > 0.f)  // as in launch_linearize_into
    return launch_pair_k<kFuseGate>(fs, accum, r64, tb, te, stride, poses, nullptr, part, pp,
                                    kappa, st);
  return launch_pair_k<kFuse32>(fs, accum, r64, tb, te, stride, poses, k, part, pp, 0.f, st);
}

hipError_t launch_reduce_pair(const vgicp_factorset_s *fs, int64_t f0, int64_t nf, double *H,
                              double *b, double *e, int64_t *inl, hipStream_t st) {
  if (nf <= 0) return hipSuccess;
  k_reduce_pair<<<unsigned(nf), 64, 0, st>>>(fs->d_factors, f0, fs->d_partials,
                                              fs->d_partials_pair, H, b, e, inl);
  return hipGetLastError();
}

hipError_t launch_overlap(const vgicp_factorset_s *fs, int64_t tb, int64_t te,
                          const double *poses, hipStream_t st, int32_t stride) {
  if (te <= tb) return hipSuccess;
  k_overlap<<<tile_grid(te - tb, fs->persist_blocks), kBlock, 0, st>>>(
      fs->d_factors, fs->d_tiles, tb, te, stride, poses, fs->d_partials);
  return hipGetLastError();
}

hipError_t launch_assemble(const vgicp_factorset_s *fs, const double *H, const double *b,
                           double *Hdiag, double *bvec, double *Hoff, hipStream_t st) {
  if (fs->n_poses > 0) {
    k_assemble_diag<<<unsigned(fs->n_poses), 64, 0, st>>>(fs->d_pose_off, fs->d_pose_ent, H, b,
                                                         Hdiag, bvec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (Hoff && fs->n_pairs > 0) {
    k_assemble_pairs<<<unsigned(fs->n_pairs), 64, 0, st>>>(fs->d_pair_off, fs->d_pair_ent, H,
                                                           Hoff);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_reduce_from(const vgicp_factorset_s *fs, int64_t f0, int64_t nf,
                              const double *poses, const double *partials, int mode, double *H,
                              double *b, double *e, int64_t *inl, double *overlap,
                              hipStream_t st) {
  if (nf <= 0) return hipSuccess;
  k_reduce<<<unsigned(nf), 64, 0, st>>>(fs->d_factors, f0, poses, partials, mode, H, b, e, inl,
                                         overlap);
  return hipGetLastError();
}

hipError_t launch_reduce(const vgicp_factorset_s *fs, int64_t f0, int64_t nf, const double *poses,
                         int mode, double *H, double *b, double *e, int64_t *inl,
                         double *overlap, hipStream_t st) {
  return launch_reduce_from(fs, f0, nf, poses, fs->d_partials, mode, H, b, e, inl, overlap, st);
}

}  // namespace vgicp
