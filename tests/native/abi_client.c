/* A C client of the renderer's C ABI, built by the tests with a C compiler in
 * strict C99 against include/dpr.h and linked against libdpr.so: no Python and
 * no PyTorch in the process.
 *
 *   abi_client check        host-side calls that need no GPU (version, camera
 *                           and partition validation, allocation counters, and
 *                           device creation, which must fail cleanly without a
 *                           GPU); prints OK on success.
 *   abi_client render DIR   render the scene described in DIR/scene.txt with
 *                           bricks DIR/brick<i>.f32 (FP32) or DIR/brick<i>.f16
 *                           (FP16, raw halves) and table DIR/tf.f32:
 *                           every brick's partial frame (dpr_render_partial),
 *                           their sort-last composite (dpr_composite) and the
 *                           whole frame (dpr_render_frame), written to
 *                           DIR/partial<i>.f32, DIR/composite.f32 and
 *                           DIR/frame.f32 (W H RGBA floats, then W H depths).
 *
 * scene.txt, whitespace-separated:
 *   dims NX NY NZ
 *   camera EX EY EZ CX CY CZ UX UY UZ FOVY W H
 *   params STEP ERT MACROCELL FLAGS
 *   tf N LO HI DENSITY
 *   dtype f32|f16
 *   bricks N
 *   then per brick: LO[3] HI[3] GHOST_LO[3] GHOST_HI[3]
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dpr.h"

#define CHECK(call)                                                                                 \
  do {                                                                                              \
    const dpr_status st_ = (call);                                                                  \
    if (st_ != DPR_OK) {                                                                            \
      fprintf(stderr, "%s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #call, (int)st_, dpr_last_error()); \
      return 1;                                                                                     \
    }                                                                                               \
  } while (0)

enum { MAX_BRICKS = 64 };

static int expect(int cond, const char* what) {
  if (!cond) fprintf(stderr, "check failed: %s\n", what);
  return cond ? 0 : 1;
}

static int run_check(void) {
  int bad = 0;
  const char* v = dpr_version();
  dpr_camera cam = {{2.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 1.0}, 60.0, 64, 48};
  dpr_camera along = cam;
  const int64_t dims[3] = {16, 8, 8};
  const int64_t lo[6] = {0, 0, 0, 8, 0, 0}, hi[6] = {8, 8, 8, 16, 8, 8};
  const int32_t glo[6] = {0, 0, 0, 1, 0, 0}, ghi[6] = {1, 0, 0, 0, 0, 0}, none[6] = {0, 0, 0, 0, 0, 0};
  int64_t allocs = -1, live = -1;
  dpr_device dev = NULL;
  dpr_status st;

  printf("version %s\n", v ? v : "(null)");
  bad += expect(v != NULL && strstr(v, "gfx950") != NULL, "the version names gfx950");
  bad += expect(dpr_check_camera(&cam) == DPR_OK, "a valid camera passes");
  along.up[0] = 1.0;
  along.up[2] = 0.0;
  bad += expect(dpr_check_camera(&along) == DPR_ERR_INVALID_ARGUMENT, "an up vector along the view is rejected");
  bad += expect(dpr_check_camera(NULL) == DPR_ERR_INVALID_ARGUMENT, "a NULL camera is rejected");
  bad += expect(dpr_check_partition(dims, 2, lo, hi, glo, ghi) == DPR_OK, "two bricks with ghost layers pass");
  bad += expect(dpr_check_partition(dims, 2, lo, hi, none, none) == DPR_ERR_INVALID_ARGUMENT,
                "an interior face without a ghost layer is rejected");
  bad += expect(dpr_alloc_stats(&allocs, &live) == DPR_OK && allocs >= 0 && live >= 0 && live <= allocs,
                "allocation counters");
  st = dpr_device_create(0, NULL, &dev);
  printf("device_create %d\n", (int)st);
  if (st == DPR_OK) {
    int32_t cu = 0, wave = 0;
    bad += expect(dpr_device_info(dev, &cu, &wave) == DPR_OK && cu > 0 && wave == 64, "device info");
    printf("cu_count %d wave_size %d\n", (int)cu, (int)wave);
    dpr_device_release(dev);
  } else {
    bad += expect(st == DPR_ERR_DEVICE && dev == NULL, "without a GPU device creation reports DPR_ERR_DEVICE");
  }
  printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}

static void* read_elems(const char* path, size_t n, size_t elem) {
  FILE* f = fopen(path, "rb");
  void* p = NULL;
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path);
    return NULL;
  }
  p = malloc(n * elem);
  if (p && fread(p, elem, n, f) != n) {
    fprintf(stderr, "%s: short read\n", path);
    free(p);
    p = NULL;
  }
  fclose(f);
  return p;
}

static int write_frame(const char* path, dpr_frame fr, int w, int h) {
  const size_t px = (size_t)w * (size_t)h;
  float* rgba = (float*)malloc(px * 4 * sizeof(float));
  float* depth = (float*)malloc(px * sizeof(float));
  FILE* f = NULL;
  int rc = 1;
  if (rgba && depth && dpr_frame_read(fr, rgba, depth) == DPR_OK && (f = fopen(path, "wb")) != NULL &&
      fwrite(rgba, sizeof(float), px * 4, f) == px * 4 && fwrite(depth, sizeof(float), px, f) == px)
    rc = 0;
  if (rc) fprintf(stderr, "writing %s failed (%s)\n", path, dpr_last_error());
  if (f) fclose(f);
  free(rgba);
  free(depth);
  return rc;
}

struct scene {
  int64_t dims[3];
  dpr_camera cam;
  dpr_render_params prm;
  int tf_n;
  float tf_lo, tf_hi, density;
  int f16;
  int n;
  int64_t lo[MAX_BRICKS][3], hi[MAX_BRICKS][3];
  int32_t glo[MAX_BRICKS][3], ghi[MAX_BRICKS][3];
};

static int read_scene(const char* dir, struct scene* s) {
  char path[4096];
  FILE* f;
  long long d[3];
  int i, a, ok;
  snprintf(path, sizeof path, "%s/scene.txt", dir);
  f = fopen(path, "r");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path);
    return 1;
  }
  ok = fscanf(f, " dims %lld %lld %lld", &d[0], &d[1], &d[2]) == 3;
  for (a = 0; a < 3; ++a) s->dims[a] = d[a];
  ok = ok && fscanf(f, " camera %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %d %d", &s->cam.eye[0], &s->cam.eye[1],
                    &s->cam.eye[2], &s->cam.center[0], &s->cam.center[1], &s->cam.center[2], &s->cam.up[0],
                    &s->cam.up[1], &s->cam.up[2], &s->cam.fovy_deg, &s->cam.width, &s->cam.height) == 12;
  ok = ok && fscanf(f, " params %f %f %d %u", &s->prm.step_voxels, &s->prm.ert_threshold, &s->prm.macrocell_cells,
                    &s->prm.flags) == 4;
  ok = ok && fscanf(f, " tf %d %f %f %f", &s->tf_n, &s->tf_lo, &s->tf_hi, &s->density) == 4;
  {
    char dt[8] = {0};
    ok = ok && fscanf(f, " dtype %7s", dt) == 1 && (strcmp(dt, "f32") == 0 || strcmp(dt, "f16") == 0);
    s->f16 = strcmp(dt, "f16") == 0;
  }
  ok = ok && fscanf(f, " bricks %d", &s->n) == 1 && s->n >= 1 && s->n <= MAX_BRICKS;
  for (i = 0; ok && i < s->n; ++i) {
    long long v[6];
    int g[6];
    ok = fscanf(f, " %lld %lld %lld %lld %lld %lld %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                &g[0], &g[1], &g[2], &g[3], &g[4], &g[5]) == 12;
    for (a = 0; ok && a < 3; ++a) {
      s->lo[i][a] = v[a];
      s->hi[i][a] = v[3 + a];
      s->glo[i][a] = g[a];
      s->ghi[i][a] = g[3 + a];
    }
  }
  fclose(f);
  if (!ok) fprintf(stderr, "%s: malformed\n", path);
  return ok ? 0 : 1;
}

static int run_render(const char* dir) {
  static struct scene s;
  char path[4096];
  dpr_device dev = NULL;
  dpr_world w = NULL;
  dpr_frame parts[MAX_BRICKS] = {NULL};
  dpr_frame comp = NULL, whole = NULL;
  int32_t ids[MAX_BRICKS];
  int64_t allocs0 = 0, live0 = 0, allocs1 = 0, live1 = 0;
  float* tf;
  int i, a;
  if (read_scene(dir, &s)) return 1;
  snprintf(path, sizeof path, "%s/tf.f32", dir);
  tf = (float*)read_elems(path, (size_t)s.tf_n * 4, sizeof(float));
  if (!tf) return 1;
  CHECK(dpr_alloc_stats(&allocs0, &live0));
  CHECK(dpr_device_create(0, NULL, &dev));
  CHECK(dpr_world_create(dev, s.dims, &w));
  CHECK(dpr_set_render_params(w, &s.prm));
  for (i = 0; i < s.n; ++i) {
    size_t nv = 1;
    int32_t id = -1;
    void* vox;
    for (a = 0; a < 3; ++a) nv *= (size_t)(s.hi[i][a] - s.lo[i][a] + s.glo[i][a] + s.ghi[i][a]);
    snprintf(path, sizeof path, "%s/brick%d.%s", dir, i, s.f16 ? "f16" : "f32");
    vox = read_elems(path, nv, s.f16 ? 2 : 4);
    if (!vox) return 1;
    /* host memory: the library copies the stored region and the buffer is freed at once */
    CHECK(dpr_world_add_brick(w, vox, s.f16 ? DPR_F16 : DPR_F32, 0, s.lo[i], s.hi[i], s.glo[i], s.ghi[i], &id));
    free(vox);
    if (id != i) {
      fprintf(stderr, "brick %d got id %d\n", i, (int)id);
      return 1;
    }
    ids[i] = id;
  }
  CHECK(dpr_world_commit(w));
  CHECK(dpr_set_transfer_function(w, tf, s.tf_n, s.tf_lo, s.tf_hi, s.density));
  free(tf);
  CHECK(dpr_set_camera(w, &s.cam));
  for (i = 0; i < s.n; ++i) {
    CHECK(dpr_frame_create(dev, s.cam.width, s.cam.height, &parts[i]));
    CHECK(dpr_render_partial(w, i, parts[i]));
    snprintf(path, sizeof path, "%s/partial%d.f32", dir, i);
    if (write_frame(path, parts[i], s.cam.width, s.cam.height)) return 1;
  }
  CHECK(dpr_frame_create(dev, s.cam.width, s.cam.height, &comp));
  CHECK(dpr_composite(dev, parts, ids, s.n, comp));
  snprintf(path, sizeof path, "%s/composite.f32", dir);
  if (write_frame(path, comp, s.cam.width, s.cam.height)) return 1;
  CHECK(dpr_frame_create(dev, s.cam.width, s.cam.height, &whole));
  CHECK(dpr_render_frame(w, whole));
  snprintf(path, sizeof path, "%s/frame.f32", dir);
  if (write_frame(path, whole, s.cam.width, s.cam.height)) return 1;
  for (i = 0; i < s.n; ++i) dpr_frame_release(parts[i]);
  dpr_frame_release(comp);
  dpr_frame_release(whole);
  dpr_world_release(w);
  dpr_device_release(dev);
  CHECK(dpr_alloc_stats(&allocs1, &live1));
  printf("allocations %lld, live before %lld after %lld\n", (long long)(allocs1 - allocs0), (long long)live0,
         (long long)live1);
  if (live1 != live0) {
    fprintf(stderr, "%lld allocations left behind\n", (long long)(live1 - live0));
    return 1;
  }
  printf("OK\n");
  return 0;
}

int main(int argc, char** argv) {
  if (argc == 2 && strcmp(argv[1], "check") == 0) return run_check();
  if (argc == 3 && strcmp(argv[1], "render") == 0) return run_render(argv[2]);
  fprintf(stderr, "usage: %s check | render DIR\n", argv[0]);
  return 2;
}
