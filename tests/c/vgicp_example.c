/* A plain C client of the C ABI in include/vgicp.h (no PyTorch, no Python).
 *
 *   vgicp_example                    checks that need no device: version,
 *                                    factor validation, NULL handling, and a
 *                                    context on a device that does not exist
 *   vgicp_example <in.bin> <out.bin> one factor on device 0: voxelize the
 *                                    target, bind the factor, linearize it at
 *                                    the given poses and evaluate its overlap
 *
 * in.bin:  int64 n_src, n_tgt; double resolution; double poses[2][12];
 *          float src_xyz[3][n_src], src_cov[n_src][6], tgt_xyz[3][n_tgt],
 *          tgt_cov[n_tgt][6]
 * out.bin: double H[144], b[12], e; int64 inliers, hits; double overlap
 *
 * Device memory comes from hipMalloc; every call's status is checked and a
 * failure prints the library's message and exits nonzero. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vgicp.h"

#define CHECK(call)                                                                 \
  do {                                                                              \
    int rc_ = (call);                                                               \
    if (rc_ != VGICP_OK) {                                                          \
      fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, vgicp_last_error(ctx));  \
      return 1;                                                                     \
    }                                                                               \
  } while (0)

#define HIP_CHECK(call)                                                             \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));             \
      return 1;                                                                     \
    }                                                                               \
  } while (0)

static int no_device_checks(void) {
  vgicp_ctx ctx = NULL;
  if (vgicp_version() <= 0) return fprintf(stderr, "bad version\n"), 1;
  if (!vgicp_last_error(NULL)) return fprintf(stderr, "NULL message\n"), 1;
  vgicp_factor good[2] = {{0, 0, 0, 1}, {1, 0, 1, 0}};
  vgicp_factor bad[1] = {{0, 2, 0, 1}};
  if (vgicp_validate_factors(2, 1, 2, good, 2) != VGICP_OK) return fprintf(stderr, "good\n"), 1;
  if (vgicp_validate_factors(2, 1, 2, bad, 1) != VGICP_EINVAL) return fprintf(stderr, "bad\n"), 1;
  if (vgicp_voxelize(NULL, NULL, 0.5, NULL) != VGICP_EINVAL) return fprintf(stderr, "null\n"), 1;
  if (vgicp_ctx_create(4096, NULL, &ctx) == VGICP_OK || ctx != NULL)
    return fprintf(stderr, "context on a missing device\n"), 1;
  printf("no-device checks ok (version %d)\n", vgicp_version());
  return 0;
}

static void *read_all(const char *path, size_t *size) {
  FILE *f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  void *buf = malloc((size_t)n);
  if (buf && fread(buf, 1, (size_t)n, f) != (size_t)n) {
    free(buf);
    buf = NULL;
  }
  fclose(f);
  *size = (size_t)n;
  return buf;
}

static int run_factor(const char *in_path, const char *out_path) {
  vgicp_ctx ctx = NULL;
  size_t size = 0;
  char *in = (char *)read_all(in_path, &size);
  if (!in) return fprintf(stderr, "cannot read %s\n", in_path), 1;
  int64_t n_src, n_tgt;
  double resolution, poses[24];
  memcpy(&n_src, in, 8);
  memcpy(&n_tgt, in + 8, 8);
  memcpy(&resolution, in + 16, 8);
  memcpy(poses, in + 24, sizeof(poses));
  const size_t head = 24 + sizeof(poses);
  const size_t want = head + (size_t)(n_src + n_tgt) * 9 * sizeof(float);
  if (size != want) return fprintf(stderr, "bad input size\n"), 1;
  const float *h_src = (const float *)(in + head);
  const float *h_tgt = h_src + 9 * n_src;

  CHECK(vgicp_ctx_create(0, NULL, &ctx));
  float *d_sx = NULL, *d_sc = NULL, *d_tx = NULL, *d_tc = NULL;
  double *d_poses = NULL, *d_out = NULL;
  int64_t *d_cnt = NULL;
  HIP_CHECK(hipMalloc((void **)&d_sx, (size_t)n_src * 3 * sizeof(float)));
  HIP_CHECK(hipMalloc((void **)&d_sc, (size_t)n_src * 6 * sizeof(float)));
  HIP_CHECK(hipMalloc((void **)&d_tx, (size_t)n_tgt * 3 * sizeof(float)));
  HIP_CHECK(hipMalloc((void **)&d_tc, (size_t)n_tgt * 6 * sizeof(float)));
  HIP_CHECK(hipMalloc((void **)&d_poses, sizeof(poses)));
  HIP_CHECK(hipMalloc((void **)&d_out, 158 * sizeof(double)));
  HIP_CHECK(hipMalloc((void **)&d_cnt, 2 * sizeof(int64_t)));
  HIP_CHECK(hipMemcpy(d_sx, h_src, (size_t)n_src * 3 * sizeof(float), hipMemcpyHostToDevice));
  HIP_CHECK(hipMemcpy(d_sc, h_src + 3 * n_src, (size_t)n_src * 6 * sizeof(float),
                      hipMemcpyHostToDevice));
  HIP_CHECK(hipMemcpy(d_tx, h_tgt, (size_t)n_tgt * 3 * sizeof(float), hipMemcpyHostToDevice));
  HIP_CHECK(hipMemcpy(d_tc, h_tgt + 3 * n_tgt, (size_t)n_tgt * 6 * sizeof(float),
                      hipMemcpyHostToDevice));
  HIP_CHECK(hipMemcpy(d_poses, poses, sizeof(poses), hipMemcpyHostToDevice));

  /* clouds: xyz planes [3][n] and covariances [n][6] */
  vgicp_cloud src = {d_sx, d_sc, n_src};
  vgicp_cloud tgt = {d_tx, d_tc, n_tgt};
  vgicp_map map = NULL;
  CHECK(vgicp_voxelize(ctx, &tgt, resolution, &map));
  vgicp_factor factor = {0, 0, 0, 1}; /* source 0 against map 0, poses i = 0, j = 1 */
  vgicp_factorset fs = NULL;
  CHECK(vgicp_factorset_create(ctx, &src, 1, &map, 1, &factor, 1, 2, 0, &fs));
  vgicp_opts opts;
  memset(&opts, 0, sizeof(opts)); /* the defaults: compensated FP32 accumulation, batched,
                                    FP64 residual, FP64 fused covariance */
  CHECK(vgicp_linearize_factors(ctx, fs, d_poses, &opts, d_out, d_out + 144, d_out + 156,
                                d_cnt, NULL));
  CHECK(vgicp_overlap(ctx, fs, d_poses, d_cnt + 1, d_out + 157));
  CHECK(vgicp_ctx_synchronize(ctx));

  double out_d[158];
  int64_t out_i[2];
  HIP_CHECK(hipMemcpy(out_d, d_out, sizeof(out_d), hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemcpy(out_i, d_cnt, sizeof(out_i), hipMemcpyDeviceToHost));
  FILE *f = fopen(out_path, "wb");
  if (!f) return fprintf(stderr, "cannot write %s\n", out_path), 1;
  fwrite(out_d, sizeof(double), 157, f);
  fwrite(out_i, sizeof(int64_t), 2, f);
  fwrite(&out_d[157], sizeof(double), 1, f);
  fclose(f);
  printf("factor ok: inliers %lld, hits %lld, e %.6e\n", (long long)out_i[0],
         (long long)out_i[1], out_d[156]);

  CHECK(vgicp_factorset_destroy(fs));
  CHECK(vgicp_map_free(map));
  CHECK(vgicp_ctx_destroy(ctx));
  hipFree(d_sx);
  hipFree(d_sc);
  hipFree(d_tx);
  hipFree(d_tc);
  hipFree(d_poses);
  hipFree(d_out);
  hipFree(d_cnt);
  free(in);
  return 0;
}

int main(int argc, char **argv) {
  if (argc == 1) return no_device_checks();
  if (argc == 3) return run_factor(argv[1], argv[2]);
  fprintf(stderr, "usage: %s [in.bin out.bin]\n", argv[0]);
  return 2;
}
