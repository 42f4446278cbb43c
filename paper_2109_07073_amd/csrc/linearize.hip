// VGICP factor linearization, cost evaluation and overlap on gfx950.
//
// Paper: Sec. III-A, Eqs. (2)-(6) (Hessian factor of one matching-cost
// factor) and Sec. III-B, Eqs. (7)-(8) (overlap).  The sums of Eqs. (3), (5)
// and (6) are reduced without atomics: every workgroup tile writes one
// partial, and a second kernel adds a factor's partials in a fixed order.
//
// Per-point work is 3x3 algebra, not a dense contraction, so everything runs
// on the vector ALUs in FP32; only the final per-factor sums are FP64.
//
// Source-frame form.  With T = T_j^-1 T_i = (R, t) and the right perturbation
// of T_i, A_k = R [[mu]x, -I], so A^T Omega A = J'^T Omega' J' with
// J' = [[mu]x, -I] and Omega' = R^T Omega R = (R^T C'_k R + C_k)^-1.  Each
// point therefore adds to a symmetric 6x6 (21 sums), a 6-vector and the cost:
// 28 sums instead of the 78 + 12 + 1 of the 12x12 system.  The remaining
// blocks follow exactly from B_k = -A_k Ad(T^-1):
//   H_ij = -H_ii Ad,  H_jj = Ad^T H_ii Ad,  b_j = -Ad^T b_i,
// which the reduce kernel applies once per factor in FP64.

#include "vgicp_internal.hpp"

namespace vgicp {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------- poses
// T_j^-1 T_i in FP64 with a fixed evaluation order and no contraction, and
// exactly (I, 0) for bitwise-equal poses.  The FP32 rounding of this pose
// drives the correspondence decision, so its order is part of the contract.
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

// The FP32 transform that decides correspondences, evaluated without fused
// multiply-add in a fixed order.
__device__ __forceinline__ void lookup_transform(const float R[9], const float t[3], float x,
                                                 float y, float z, float q[3]) {
#pragma clang fp contract(off)
  q[0] = ((R[0] * x + R[1] * y) + R[2] * z) + t[0];
  q[1] = ((R[3] * x + R[4] * y) + R[5] * z) + t[1];
  q[2] = ((R[6] * x + R[7] * y) + R[8] * z) + t[2];
}

// Global-address-space views: loads through them compile to global_load_*
// (flat loads would also tie up the LDS counter).
typedef const float __attribute__((address_space(1))) gfloat;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const f32x4 __attribute__((address_space(1))) gfloat4;
typedef const uint64_t __attribute__((address_space(1))) gu64;

// One source point: position and covariance (xx xy xz yy yz zz).
struct SrcPoint {
  float x, y, z;
  float c[6];
};

template <bool COV>
__device__ __forceinline__ void load_point(const float *px, const float *pc, int64_t n, int64_t i,
                                           SrcPoint &p) {
  gfloat *gx = (gfloat *)px;
  p.x = __builtin_nontemporal_load(gx + i);
  p.y = __builtin_nontemporal_load(gx + n + i);
  p.z = __builtin_nontemporal_load(gx + 2 * n + i);
  if constexpr (COV) {
    gfloat *gc = (gfloat *)pc;
#pragma unroll
    for (int a = 0; a < 6; ++a) p.c[a] = __builtin_nontemporal_load(gc + a * n + i);
  }
}

// Packed key and home slot of the voxel holding q (ok = false when a key
// would fall outside [-2^20, 2^20), which no voxel of any map has).
struct VoxelKey {
  bool ok;
  uint64_t key;
  uint32_t h;
};

__device__ __forceinline__ VoxelKey voxel_key(const float q[3], float s, uint32_t log2cap) {
  const float vx = q[0] * s, vy = q[1] * s, vz = q[2] * s;
  VoxelKey r;
  r.ok = (vx >= -kKeyLimitF) & (vx < kKeyLimitF) & (vy >= -kKeyLimitF) & (vy < kKeyLimitF) &
         (vz >= -kKeyLimitF) & (vz < kKeyLimitF);
  r.key = r.ok ? pack_key(int32_t(floorf(vx)), int32_t(floorf(vy)), int32_t(floorf(vz))) : 0;
  r.h = hash_slot(r.key, log2cap);
  return r;
}

// The first 48 bytes of a slot: key (w0.xy), mean (w0.zw, w1.x), covariance
// (w1.yzw, w2.xyz), ordinal (w2.w).
struct SlotData {
  f32x4 w0, w1, w2;
};

__device__ __forceinline__ void load_slot(const Slot *slots, uint32_t h, SlotData &d) {
  gfloat4 *p = (gfloat4 *)(slots + h);
  d.w0 = p[0];
  d.w1 = p[1];
  d.w2 = p[2];
}

__device__ __forceinline__ uint64_t slot_key(const SlotData &d) {
  return (uint64_t(__float_as_uint(d.w0.y)) << 32) | uint64_t(__float_as_uint(d.w0.x));
}

// Linear probing from a speculatively loaded home slot: true when `key` is
// found (d then holds its slot), false at the first empty slot.  At most
// `capacity` slots are visited.
__device__ __forceinline__ bool resolve_slot(const Slot *slots, uint32_t log2cap, uint64_t key,
                                             uint32_t h, SlotData &d) {
  uint64_t k = slot_key(d);
  if (k != key && k != kEmptyKey) {
    // Rare: keep probing.  The full wait at the end leaves no slot load in
    // flight on this path, so the common path's waits stay exact (they only
    // need the home slot, not the prefetched next point).
    const uint32_t mask = (1u << log2cap) - 1u;
    for (uint32_t p = 0; p < mask; ++p) {
      h = (h + 1u) & mask;
      load_slot(slots, h, d);
      k = slot_key(d);
      if (k == key || k == kEmptyKey) break;
    }
    __builtin_amdgcn_s_waitcnt(0);
  }
  return k == key;
}

// Key-only probing for the overlap count.
__device__ __forceinline__ bool contains_key(const Slot *slots, uint32_t log2cap, uint64_t key,
                                             uint32_t h) {
  const uint32_t mask = (1u << log2cap) - 1u;
  for (uint32_t p = 0; p <= mask; ++p) {
    const uint64_t k = *(gu64 *)(&slots[h].key);
    if (k == key) return true;
    if (k == kEmptyKey) return false;
    h = (h + 1u) & mask;
  }
  return false;
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

// Rounding error of the FP32 lookup transform against the exact relative
// motion: (R mu + t) - q with q the FP32 transform of lookup_transform,
// accurate to a few units in the last place of the error itself.  Products
// are split exactly with fma, the fixed-order sums with two-sum, and the
// FP32 rounding of R and t enters through their low parts.  q itself is the
// high part of this double-float evaluation, so the correspondence decision
// is unchanged.
__device__ __forceinline__ void transform_error(const float R[9], const float Rlo[9],
                                                const float t[3], const float tlo[3], float x,
                                                float y, float z, float qerr[3]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float p0 = R[3 * r] * x, p1 = R[3 * r + 1] * y, p2 = R[3 * r + 2] * z;
    const float e0 = __builtin_fmaf(R[3 * r], x, -p0);
    const float e1 = __builtin_fmaf(R[3 * r + 1], y, -p1);
    const float e2 = __builtin_fmaf(R[3 * r + 2], z, -p2);
    float s1, s2, s3, d1, d2, d3;
    two_sum(p0, p1, s1, d1);
    two_sum(s1, p2, s2, d2);
    two_sum(s2, t[r], s3, d3);
    const float lo = __builtin_fmaf(Rlo[3 * r], x, __builtin_fmaf(Rlo[3 * r + 1], y,
                                                                  Rlo[3 * r + 2] * z));
    qerr[r] = ((e0 + e1) + (e2 + d1)) + ((d2 + d3) + (tlo[r] + lo));
  }
}

template <int N>
struct Sums<VGICP_ACC_F32_COMP, N> {
  float v[N];
  float c[N];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = c[i] = 0.f;
  }
  __device__ __forceinline__ void add(int i, float x) {
    float s, err;
    two_sum(v[i], x, s, err);
    v[i] = s;
    c[i] += err;
  }
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
      step<0xb1>(v[i], c[i]);
      step<0x4e>(v[i], c[i]);
      step<0x141>(v[i], c[i]);
      step<0x140>(v[i], c[i]);
      step<0x142, 0xa>(v[i], c[i]);
      step<0x143, 0xc>(v[i], c[i]);
    }
  }
  __device__ void store(double *lds, int wave) const {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[wave * N + i] = double(v[i]) + double(c[i]);
  }
  using lds_t = double;
  __device__ static double finish(const double *lds, int i) {
    double s = lds[i];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += lds[w * N + i];
    return s;
  }
};

// ---------------------------------------------------------------- per point
// Adds one correspondence.  R is the FP32 relative rotation, (mx, my, mz) the
// source point, c its covariance, q its FP32 transform, m / S the voxel mean
// and covariance.  With LIN the 21 + 6 source-frame Hessian/gradient sums and
// the cost are added; without it only the cost.
template <bool LIN, typename SumsT>
__device__ __forceinline__ void add_correspondence(SumsT &acc, const float R[9], float mx,
                                                   float my, float mz, const float c[6],
                                                   const float q[3], const float qerr[3],
                                                   const float m[3], const float S[6]) {
  // residual e_k = mu' - T mu (target frame), rotated into the source frame;
  // m - q is exact when the two are within a factor of two, and qerr carries
  // the transform's rounding error (zero for the plain FP32 residual)
  const float e0 = (m[0] - q[0]) - qerr[0];
  const float e1 = (m[1] - q[1]) - qerr[1];
  const float e2 = (m[2] - q[2]) - qerr[2];
  const float r0 = R[0] * e0 + R[3] * e1 + R[6] * e2;
  const float r1 = R[1] * e0 + R[4] * e1 + R[7] * e2;
  const float r2 = R[2] * e0 + R[5] * e1 + R[8] * e2;
  // W = C' R, then F' = R^T W + C (symmetric, upper triangle)
  const float W00 = S[0] * R[0] + S[1] * R[3] + S[2] * R[6];
  const float W01 = S[0] * R[1] + S[1] * R[4] + S[2] * R[7];
  const float W02 = S[0] * R[2] + S[1] * R[5] + S[2] * R[8];
  const float W10 = S[1] * R[0] + S[3] * R[3] + S[4] * R[6];
  const float W11 = S[1] * R[1] + S[3] * R[4] + S[4] * R[7];
  const float W12 = S[1] * R[2] + S[3] * R[5] + S[4] * R[8];
  const float W20 = S[2] * R[0] + S[4] * R[3] + S[5] * R[6];
  const float W21 = S[2] * R[1] + S[4] * R[4] + S[5] * R[7];
  const float W22 = S[2] * R[2] + S[4] * R[5] + S[5] * R[8];
  const float f00 = (R[0] * W00 + R[3] * W10 + R[6] * W20) + c[0];
  const float f01 = (R[0] * W01 + R[3] * W11 + R[6] * W21) + c[1];
  const float f02 = (R[0] * W02 + R[3] * W12 + R[6] * W22) + c[2];
  const float f11 = (R[1] * W01 + R[4] * W11 + R[7] * W21) + c[3];
  const float f12 = (R[1] * W02 + R[4] * W12 + R[7] * W22) + c[4];
  const float f22 = (R[2] * W02 + R[5] * W12 + R[8] * W22) + c[5];
  // Omega' = F'^-1 by the adjugate
  const float a00 = f11 * f22 - f12 * f12;
  const float a01 = f02 * f12 - f01 * f22;
  const float a02 = f01 * f12 - f02 * f11;
  const float a11 = f00 * f22 - f02 * f02;
  const float a12 = f01 * f02 - f00 * f12;
  const float a22 = f00 * f11 - f01 * f01;
  const float det = f00 * a00 + f01 * a01 + f02 * a02;
  if (!((f00 > 0.f) & (a22 > 0.f) & (det > 0.f))) return;  // not positive definite
  const float inv = 1.0f / det;
  const float o00 = a00 * inv, o01 = a01 * inv, o02 = a02 * inv;
  const float o11 = a11 * inv, o12 = a12 * inv, o22 = a22 * inv;
  // g = Omega' r
  const float g0 = o00 * r0 + o01 * r1 + o02 * r2;
  const float g1 = o01 * r0 + o11 * r1 + o12 * r2;
  const float g2 = o02 * r0 + o12 * r1 + o22 * r2;
  acc.add(LIN ? 27 : 0, r0 * g0 + r1 * g1 + r2 * g2);
  if constexpr (LIN) {
    // M = [mu]x Omega' (column c = mu x Omega'_c): the (omega, rho) block
    const float M00 = my * o02 - mz * o01, M10 = mz * o00 - mx * o02, M20 = mx * o01 - my * o00;
    const float M01 = my * o12 - mz * o11, M11 = mz * o01 - mx * o12, M21 = mx * o11 - my * o01;
    const float M02 = my * o22 - mz * o12, M12 = mz * o02 - mx * o22, M22 = mx * o12 - my * o02;
    // (omega, omega) block [mu]x^T Omega' [mu]x, row r = mu x (row r of M)
    acc.add(0, my * M02 - mz * M01);
    acc.add(1, mz * M00 - mx * M02);
    acc.add(2, mx * M01 - my * M00);
    acc.add(3, M00);
    acc.add(4, M01);
    acc.add(5, M02);
    acc.add(6, mz * M10 - mx * M12);
    acc.add(7, mx * M11 - my * M10);
    acc.add(8, M10);
    acc.add(9, M11);
    acc.add(10, M12);
    acc.add(11, mx * M21 - my * M20);
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
    acc.add(21, g1 * mz - g2 * my);
    acc.add(22, g2 * mx - g0 * mz);
    acc.add(23, g0 * my - g1 * mx);
    acc.add(24, -g0);
    acc.add(25, -g1);
    acc.add(26, -g2);
  }
}

// ---------------------------------------------------------------- tiles
// Map a block to a tile so that each XCD (blocks are dealt round-robin over
// the 8 XCDs) works through one contiguous range of the tile table: tiles of
// one factor, and factors sorted by target map, then share that XCD's L2.
__device__ __forceinline__ int64_t block_tile(int64_t tile_base) {
  const uint32_t per = gridDim.x >> 3;  // the grid is a multiple of 8
  return tile_base + int64_t(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
}

struct FactorConsts {
  float R[9];    // fl32(R)
  float t[3];    // fl32(t)
  float Rlo[9];  // fl32(R - fl32(R))
  float tlo[3];  // fl32(t - fl32(t))
};

__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ FactorConsts factor_consts(const FactorDesc &fd,
                                                      const double *__restrict__ poses) {
  double R[9], t[3];
  relative_pose64(poses + 12 * int64_t(fd.pose_i), poses + 12 * int64_t(fd.pose_j), R, t);
  FactorConsts k;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    k.R[i] = uniform_f(float(R[i]));
    k.Rlo[i] = uniform_f(float(R[i] - double(k.R[i])));
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    k.t[i] = uniform_f(float(t[i]));
    k.tlo[i] = uniform_f(float(t[i] - double(k.t[i])));
  }
  return k;
}

// Linearization (LIN) or cost evaluation (!LIN) of one tile per block.
// FF: residual from the double-float transform (else plain FP32).
template <int ACC, bool LIN, bool FF>
__global__ void __launch_bounds__(kBlock)
k_linearize(const FactorDesc *__restrict__ factors, const Tile *__restrict__ tiles,
            int64_t tile_base, int64_t tile_end, int32_t tile_points,
            const double *__restrict__ poses, double *__restrict__ partials,
            int32_t *__restrict__ corr) {
  constexpr int N = LIN ? kNumSums : 1;
  using SumsT = Sums<ACC, N>;
  __shared__ typename SumsT::lds_t lds[kWaves * N];
  __shared__ int lds_cnt[kWaves];

  const int64_t tile = block_tile(tile_base);
  if (tile >= tile_end) return;
  const Tile td = tiles[tile];
  const FactorDesc fd = factors[td.factor];
  const FactorConsts k = factor_consts(fd, poses);
  const int64_t n = fd.n;
  const float *__restrict__ px = fd.xyz;
  const float *__restrict__ pc = fd.cov;
  const Slot *__restrict__ slots = fd.slots;
  const int64_t begin = td.start;
  const int64_t end = min(begin + int64_t(tile_points), n);
  int32_t *__restrict__ pcorr = corr ? corr + fd.corr_offset : nullptr;

  SumsT acc;
  acc.zero();
  int inl = 0;
  // Software pipeline: the next point's HBM loads are issued after the
  // current point's slot load, so they are in flight during the lookup and
  // the math (vector loads return in order, so the slot can be waited for
  // without waiting for the prefetch).
  SrcPoint cur, nxt;
  int64_t i = begin + threadIdx.x;
  if (i < end) load_point<true>(px, pc, n, i, cur);
  for (; i < end; i += kBlock) {
    float q[3];
    lookup_transform(k.R, k.t, cur.x, cur.y, cur.z, q);
    const VoxelKey vk = voxel_key(q, fd.scale, fd.log2cap);
    // Both loads are unconditional (an out-of-range key reads its hash slot,
    // the last iteration re-reads the tile's last point) so that the wait for
    // the slot leaves exactly the nine prefetch loads in flight.
    SlotData d;
    load_slot(slots, vk.h, d);
    load_point<true>(px, pc, n, min(i + kBlock, end - 1), nxt);
    const bool hit = vk.ok && resolve_slot(slots, fd.log2cap, vk.key, vk.h, d);
    if (pcorr) pcorr[i] = hit ? __float_as_int(d.w2.w) : -1;
    if (hit) {
      ++inl;
      const float m[3] = {d.w0.z, d.w0.w, d.w1.x};
      const float S[6] = {d.w1.y, d.w1.z, d.w1.w, d.w2.x, d.w2.y, d.w2.z};
      float qerr[3] = {0.f, 0.f, 0.f};
      if constexpr (FF) transform_error(k.R, k.Rlo, k.t, k.tlo, cur.x, cur.y, cur.z, qerr);
      add_correspondence<LIN>(acc, k.R, cur.x, cur.y, cur.z, cur.c, q, qerr, m, S);
    }
    cur = nxt;
  }

  acc.wave_reduce();
  inl = wave_sum(inl);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == kLastLane) {
    acc.store(lds, wave);
    lds_cnt[wave] = inl;
  }
  __syncthreads();
  double *__restrict__ out = partials + tile * kPartialStride;
  if (threadIdx.x < N) {
    out[LIN ? threadIdx.x : 27] = SumsT::finish(lds, threadIdx.x);
  } else if (threadIdx.x == 32) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += lds_cnt[w];
    out[kNumSums] = double(s);
  }
}

// Overlap hit counts of one tile per block (Eq. (7)).
__global__ void __launch_bounds__(kBlock)
k_overlap(const FactorDesc *__restrict__ factors, const Tile *__restrict__ tiles,
          int64_t tile_base, int64_t tile_end, int32_t tile_points,
          const double *__restrict__ poses, double *__restrict__ partials) {
  __shared__ int lds_cnt[kWaves];
  const int64_t tile = block_tile(tile_base);
  if (tile >= tile_end) return;
  const Tile td = tiles[tile];
  const FactorDesc fd = factors[td.factor];
  const FactorConsts k = factor_consts(fd, poses);
  const int64_t n = fd.n;
  const float *__restrict__ px = fd.xyz;
  const int64_t begin = td.start;
  const int64_t end = min(begin + int64_t(tile_points), n);
  int hits = 0;
  SrcPoint cur, nxt;
  int64_t i = begin + threadIdx.x;
  if (i < end) load_point<false>(px, nullptr, n, i, cur);
  for (; i < end; i += kBlock) {
    float q[3];
    lookup_transform(k.R, k.t, cur.x, cur.y, cur.z, q);
    const VoxelKey vk = voxel_key(q, fd.scale, fd.log2cap);
    load_point<false>(px, nullptr, n, min(i + kBlock, end - 1), nxt);
    hits += vk.ok && contains_key(fd.slots, fd.log2cap, vk.key, vk.h);
    cur = nxt;
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
        acc += partials[int64_t(fd.tile_begin + tt) * kPartialStride + lane];
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

// ---------------------------------------------------------------- launchers
static inline unsigned xcd_grid(int64_t tiles) { return unsigned(((tiles + 7) / 8) * 8); }

template <int ACC, bool LIN, bool FF>
static hipError_t launch_lin(const vgicp_factorset_s *fs, int64_t tb, int64_t te,
                             const double *poses, int32_t *corr, hipStream_t st) {
  if (te <= tb) return hipSuccess;
  k_linearize<ACC, LIN, FF><<<xcd_grid(te - tb), kBlock, 0, st>>>(
      fs->d_factors, fs->d_tiles, tb, te, fs->tile_points, poses, fs->d_partials, corr);
  return hipGetLastError();
}

template <int ACC>
static hipError_t launch_acc(const vgicp_factorset_s *fs, bool lin, bool ff, int64_t tb,
                             int64_t te, const double *poses, int32_t *corr, hipStream_t st) {
  if (lin) {
    return ff ? launch_lin<ACC, true, true>(fs, tb, te, poses, corr, st)
              : launch_lin<ACC, true, false>(fs, tb, te, poses, corr, st);
  }
  return ff ? launch_lin<ACC, false, true>(fs, tb, te, poses, corr, st)
            : launch_lin<ACC, false, false>(fs, tb, te, poses, corr, st);
}

hipError_t launch_linearize(const vgicp_factorset_s *fs, int accum, int resid, bool lin,
                            int64_t tb, int64_t te, const double *poses, int32_t *corr,
                            hipStream_t st) {
  const bool ff = resid == VGICP_RESID_FF;
  switch (accum) {
    case VGICP_ACC_F64:
      return launch_acc<VGICP_ACC_F64>(fs, lin, ff, tb, te, poses, corr, st);
    case VGICP_ACC_F32_COMP:
      return launch_acc<VGICP_ACC_F32_COMP>(fs, lin, ff, tb, te, poses, corr, st);
    default:
      return launch_acc<VGICP_ACC_F32>(fs, lin, ff, tb, te, poses, corr, st);
  }
}

hipError_t launch_overlap(const vgicp_factorset_s *fs, int64_t tb, int64_t te,
                          const double *poses, hipStream_t st) {
  if (te <= tb) return hipSuccess;
  k_overlap<<<xcd_grid(te - tb), kBlock, 0, st>>>(fs->d_factors, fs->d_tiles, tb, te,
                                                   fs->tile_points, poses, fs->d_partials);
  return hipGetLastError();
}

hipError_t launch_reduce(const vgicp_factorset_s *fs, int64_t f0, int64_t nf, const double *poses,
                         int mode, double *H, double *b, double *e, int64_t *inl,
                         double *overlap, hipStream_t st) {
  if (nf <= 0) return hipSuccess;
  k_reduce<<<unsigned(nf), 64, 0, st>>>(fs->d_factors, f0, poses, fs->d_partials, mode, H, b, e,
                                         inl, overlap);
  return hipGetLastError();
}

}  // namespace vgicp
