/*
 * dpr.h -- C ABI of the MI355X-native data-parallel volume renderer and
 * sort-last compositor.
 *
 * The calls follow the data-parallel rendering paradigm of "Standardized
 * Data-Parallel Rendering Using ANARI" (arXiv 2407.00179):
 *   - world content (bricks) is local to a rank and added piece by piece
 *     (section 3.1.2, Locally Defined Objects);
 *   - camera and renderer parameters are global and identical for every brick
 *     (section 3.1.1, Globally Consistent Objects);
 *   - rendering a frame is the one collective step: every local piece is
 *     rendered to an RGBA-z fragment per pixel and the fragments are composited
 *     in per-pixel depth order (section 3.2, Collaborative Operations;
 *     section 5.1.1, Compositing);
 *   - the finished frame is mapped where the caller asks for it
 *     (section 3.1.3, Locally Mapped Frame Buffers);
 *   - the partition is described by the application through per-piece bounds
 *     (section 8.2, Scene/Data Partitioning).
 * On one GPU each brick stands for one rank's share.  The local render itself
 * (emission-absorption ray marching) is not specified by the paper; its exact
 * definition is given with dpr_render_partial below.
 *
 * Conventions
 *   - Every call returns dpr_status; out-parameters are written only on
 *     success.  No C++ exception crosses the ABI.  dpr_last_error() returns a
 *     thread-local message for the last failing call on this thread.
 *   - Volumes are scalar grids of global dims (nx, ny, nz), x fastest.  Voxel
 *     (i,j,k) is the centre of cell [i,i+1)x[j,j+1)x[k,k+1); with
 *     h = 1/max(nx,ny,nz) the world box is [0,nx h]x[0,ny h]x[0,nz h].
 *   - A frame of W x H pixels is float RGBA premultiplied colour (16 B per
 *     pixel, row-major, row 0 at the top) plus float depth (4 B per pixel).
 *     An empty pixel is (0,0,0,0) at depth +inf.
 *   - Render and composite calls enqueue work on the device's HIP stream and
 *     return; HIP errors of that work surface as DPR_ERR_DEVICE at the next
 *     synchronising call (dpr_device_sync, dpr_frame_map, dpr_frame_read), the
 *     way an asynchronous render is followed by a map.
 *   - A device handle and the objects made from it are not thread-safe; the
 *     caller serialises calls on one device.
 */
#ifndef DPR_H
#define DPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DPR_OK = 0,
  DPR_ERR_INVALID_ARGUMENT = -1,
  DPR_ERR_INVALID_STATE = -2,
  DPR_ERR_OUT_OF_MEMORY = -3,
  DPR_ERR_DEVICE = -4,
  DPR_ERR_UNSUPPORTED = -5
} dpr_status;

typedef enum { DPR_F32 = 0, DPR_F16 = 1 } dpr_dtype;

/* render-parameter and call flags */
#define DPR_FLAG_NO_SKIP 0x1u    /* disable macrocell empty-space skipping          */
#define DPR_FLAG_PLAIN 0x2u      /* one plain launch per (camera, brick) + composite  */
#define DPR_FLAG_NO_GRAPH 0x4u   /* batched paths: enqueue directly, no graph replay */
/* render parameter: form voxel offsets in 64 bits for every brick (automatic for
 * bricks whose blocked array is 4 GiB or more); the results are identical.  For
 * FP16 bricks it implies DPR_FLAG_F16_HALVES, and changing it un-commits the
 * world (the next dpr_world_commit lays the bricks out again)                  */
#define DPR_FLAG_WIDE_OFFSETS 0x8u
/* render parameter read by dpr_world_commit: store the world's FP16 bricks as
 * 2-byte voxels, addressed with 64-bit offsets (automatic once some brick's
 * voxel-pair copy would reach 4 GiB), instead of 4-byte voxel pairs: half the
 * memory and half the cache lines per sample, more loads per sample; the results
 * are identical.  Changing it un-commits the world.                             */
#define DPR_FLAG_F16_HALVES 0x10u
/* batched renders (diagnostics): count how often each queue item is taken and
 * each of its fragment slots written, for dpr_batch_coverage; the render is then
 * enqueued directly (no graph replay).  The frames are the same bits.          */
#define DPR_FLAG_QUEUE_COVERAGE 0x20u

typedef struct dpr_device_t* dpr_device; /* one GPU + one HIP stream              */
typedef struct dpr_world_t* dpr_world;   /* this rank's bricks + TF + camera      */
typedef struct dpr_frame_t* dpr_frame;   /* W x H RGBA + depth (+ sample counts)  */

/* Pinhole camera: rays through pixel centres, vertical field of view fovy_deg.
 * f = normalize(center - eye), r = normalize(f x up), u = r x f,
 * d = normalize(f + x r + y u) with x = (2(px+.5)/W - 1) tan(fovy/2) W/H and
 * y = (1 - 2(py+.5)/H) tan(fovy/2).                                            */
typedef struct {
  double eye[3], center[3], up[3];
  double fovy_deg;
  int32_t width, height;
} dpr_camera;

/* step_voxels: lattice step dt = step_voxels * h, in (0, 1].
 * ert_threshold: stop a ray once 1 - T >= threshold; >= 1 disables.
 * macrocell_cells: macrocell edge in cells (power of two in [2, 64]).
 * flags: DPR_FLAG_NO_SKIP, DPR_FLAG_PLAIN, DPR_FLAG_NO_GRAPH (dpr_render_frame),
 * DPR_FLAG_WIDE_OFFSETS, DPR_FLAG_F16_HALVES, DPR_FLAG_QUEUE_COVERAGE. */
typedef struct {
  float step_voxels;
  float ert_threshold;
  int32_t macrocell_cells;
  uint32_t flags;
} dpr_render_params;

const char* dpr_last_error(void);
const char* dpr_version(void);
/* Allocation counters of this process (diagnostics, needs no GPU): `allocations`
 * = device and pinned host allocations attempted so far (the count that the
 * environment setting DPR_FAULT_INJECT=alloc:N refers to: the N-th attempt then
 * fails with DPR_ERR_OUT_OF_MEMORY), `live` = those not yet freed.  Either
 * pointer may be NULL.                                                           */
dpr_status dpr_alloc_stats(int64_t* allocations, int64_t* live);

/* ---------------------------------------------------------------- device */
/* Bind GPU `hip_device` and the HIP stream `hip_stream` (NULL: the null stream).
 * Fails with DPR_ERR_DEVICE when no such GPU is visible.                        */
dpr_status dpr_device_create(int hip_device, void* hip_stream, dpr_device* out);
dpr_status dpr_device_set_stream(dpr_device, void* hip_stream);
dpr_status dpr_device_sync(dpr_device);
/* Worlds, frames and deep frames hold a reference to their device: a released
 * device handle must not be used again, but its memory and stream binding stay
 * valid until the last world or frame created on it is released too.  The
 * library is not thread-safe: calls on one device come from one thread.         */
void dpr_device_release(dpr_device);
/* number of compute units and the wavefront size of the bound GPU */
dpr_status dpr_device_info(dpr_device, int32_t* cu_count, int32_t* wave_size);

/* ---------------------------------------------------------------- world */
dpr_status dpr_world_create(dpr_device, const int64_t global_dims[3], dpr_world* out);
void dpr_world_release(dpr_world);

/* Add one locally owned brick (section 3.1.2): global cells [owned_lo, owned_hi)
 * per axis plus ghost_lo/ghost_hi stored voxel layers outside them.  `voxels`
 * holds the stored region, dims = owned_hi - owned_lo + ghost_lo + ghost_hi,
 * x fastest, in host memory (voxels_on_device = 0) or device memory (1).  The
 * data are copied; the caller may free its buffer on return.  Every global dim
 * must be >= 2.  Ghost layers may not reach outside the global domain.
 * brick_id receives the brick's index (0, 1, ...), which is also its intrinsic
 * fragment id for compositing.  Adding a brick un-commits the world.
 * Device memory per brick: the linear copy (2 or 4 bytes per stored voxel) plus,
 * after commit, the blocked copy at 4 bytes per voxel (FP32, or FP16 stored as
 * voxel pairs: an element holds a voxel and its +x neighbour) or 2 bytes per
 * voxel (FP16 stored as halves: DPR_FLAG_F16_HALVES, or automatically when the
 * pair copy would reach 4 GiB) and the macrocell arrays.                        */
dpr_status dpr_world_add_brick(dpr_world, const void* voxels, dpr_dtype dtype, int voxels_on_device,
                               const int64_t owned_lo[3], const int64_t owned_hi[3],
                               const int32_t ghost_lo[3], const int32_t ghost_hi[3], int32_t* brick_id);

/* Validate the partition and build device data.  Owned boxes must be pairwise
 * disjoint axis-aligned boxes (each rank's data convex: the condition under
 * which one fragment per pixel composites correctly, section 2.1), and every
 * owned face interior to the global domain must carry >= 1 ghost layer
 * (samples fall up to half a step, at most half a voxel, outside the owned
 * box, and trilinear reads one voxel beyond that).  Then
 * each brick is re-tiled into 8^3-voxel blocks and its macrocell min/max
 * ranges are built (window [mc*m - 1, mc*m + mc] of owned-relative voxels), both
 * in one pass over the brick's linear copy; stream-ordered, the host does not
 * wait.
 * Gaps between bricks are allowed and render empty.                             */
dpr_status dpr_world_commit(dpr_world);

/* Free every brick's linear stored copy (the one dpr_world_add_brick made) once
 * the world is committed, so that a brick occupies only its blocked copy: 4 bytes
 * a voxel for FP32 and for FP16 voxel pairs, 2 for the FP16 2-byte layout (plus
 * 24 bytes a macrocell).  Waits for the device stream.  Afterwards
 * dpr_world_commit with nothing to rebuild returns DPR_OK at once; one that must
 * rebuild (bricks added, or the macrocell edge or the FP16 layout flags changed)
 * fails with DPR_ERR_INVALID_STATE, as does dpr_render_path when it must rebuild
 * its block majorants (after a commit or a transfer-function change).  Fails
 * with DPR_ERR_INVALID_STATE on a world that is not committed.                  */
dpr_status dpr_world_release_linear(dpr_world);

/* Transfer function: n_entries RGBA floats (host), entry i at value
 * value_lo + i (value_hi - value_lo)/(n_entries - 1); RGB is emitted colour,
 * A is normalised extinction; extinction per world unit = density_scale * A.
 * 2 <= n_entries <= 1024, value_hi > value_lo, density_scale >= 0.              */
dpr_status dpr_set_transfer_function(dpr_world, const float* rgba, int32_t n_entries, float value_lo,
                                     float value_hi, float density_scale);
/* Opaque iso-surface of the world's field, rendered together with the volume.
 * The paper draws iso-surfaces through the same data-parallel pipeline as volumes
 * (Fig. 1c, Fig. 3c, Fig. 4); section 5.1.2 asks the local render only for colour
 * and depth.  Along a ray, the sides (v >= value) of consecutive lattice samples
 * are compared at every lattice point in a brick's [t_in, t_out), so each pair is
 * tested by exactly one brick; at the first change of side the ray ends on an
 * opaque surface at the linearly interpolated crossing, lit by a headlight:
 * colour = TF colour at `value` * (ambient + diffuse * |cos|), cos between the
 * ray and the gradient of the trilinear patch there (taken as 1 where the
 * gradient is 0).  The segments before the crossing pair integrate as usual; the
 * fragment's alpha is then 1 and its depth stays the brick entry, so bricks
 * composite unchanged and a split volume gives the unsplit image.  enable = 0
 * turns it off (the other arguments are then ignored).  value must be finite,
 * ambient and diffuse >= 0.  Applies to every later render of the world.        */
dpr_status dpr_set_isosurface(dpr_world, int32_t enable, float value, float ambient, float diffuse);
/* Global camera (section 3.1.1: identical for every brick).                     */
dpr_status dpr_set_camera(dpr_world, const dpr_camera*);
dpr_status dpr_set_render_params(dpr_world, const dpr_render_params*);

/* Host-only validators (no GPU needed): the partition rules dpr_world_commit
 * applies (n bricks; lo/hi/ghost arrays hold 3 values per brick, x y z), and the
 * camera rules dpr_set_camera applies.                                          */
dpr_status dpr_check_partition(const int64_t global_dims[3], int32_t n, const int64_t* owned_lo,
                               const int64_t* owned_hi, const int32_t* ghost_lo, const int32_t* ghost_hi);
dpr_status dpr_check_camera(const dpr_camera*);

/* Read back brick info and macrocell data (host copies; synchronises).
 * ranges: float2 (min, max) per macrocell, majorant: float per macrocell, both
 * x-fastest over the brick's macrocell grid mc_dims; either pointer may be NULL.
 * The majorant reflects the current transfer function.                         */
dpr_status dpr_world_brick_macrocells(dpr_world, int32_t brick_id, int32_t mc_dims[3], float* ranges,
                                      float* majorant, size_t capacity);
dpr_status dpr_world_brick_count(dpr_world, int32_t* n);
/* Read back a committed brick's blocked copy (diagnostics; synchronises).
 * bdim = blocks per axis, elem_bytes = 4 (FP32 voxels, FP16 voxel pairs: the
 * halves of voxels x and x + 1, the last voxel of a row paired with itself) or
 * 2 (FP16 voxels).  Layout: 8^3-voxel blocks, x fastest then y then z; inside a
 * block the 9 index bits of stored voxel (i, j, k) are, from bit 0: i0 i1 j0 k0
 * j1 k1 i2 j2 k2 (i, j, k taken mod 8).  Elements of padding voxels beyond the
 * stored extents are zero.  host may be NULL (only bdim and elem_bytes are
 * returned); else capacity (bytes) must hold bdim[0] bdim[1] bdim[2] 512
 * elem_bytes.                                                                     */
dpr_status dpr_world_brick_blocked(dpr_world, int32_t brick_id, int32_t bdim[3], int32_t* elem_bytes, void* host,
                                   size_t capacity);

/* ---------------------------------------------------------------- frames */
dpr_status dpr_frame_create(dpr_device, int32_t width, int32_t height, dpr_frame* out);
/* Borrow caller buffers (device memory, 16 B and 4 B per pixel); they must
 * outlive the frame.                                                            */
dpr_status dpr_frame_wrap(dpr_device, int32_t width, int32_t height, float* rgba_dev, float* depth_dev,
                          dpr_frame* out);
/* Optional per-pixel logical-sample counts (int32, device memory, borrowed):
 * renders into this frame also store, per pixel, the number of lattice
 * segments of positive length processed before termination.  NULL detaches.   */
dpr_status dpr_frame_attach_counts(dpr_frame, int32_t* counts_dev);
/* Synchronise and return the frame's DEVICE pointers.                           */
dpr_status dpr_frame_map(dpr_frame, const float** rgba_dev, const float** depth_dev);
dpr_status dpr_frame_unmap(dpr_frame);
/* Synchronise and copy the frame to host buffers (either may be NULL).          */
dpr_status dpr_frame_read(dpr_frame, float* rgba_host, float* depth_host);
void dpr_frame_release(dpr_frame);

/* ---------------------------------------------------------------- rendering */
/* Render brick `brick_id` into `out` (one RGBA-z fragment per pixel; the
 * "local rendering" of section 5.1.2).  Definition (FP32 arithmetic, FP64 ray
 * geometry):
 *   ray/box clip against the owned box [lo h, hi h] -> [t_in, t_out], hit iff
 *   t_out > t_in; lattice segments s in [floor(t_in/dt), ceil(t_out/dt) - 1]
 *   anchored at the eye, clipped to length l_s; the field is sampled once per
 *   segment at t = (s + 1/2) dt by trilinear interpolation in global voxel-centre
 *   coordinates clamped to [0, n-1]; the TF is interpolated linearly;
 *   tau = D A l_s; C += T (1 - e^-tau) rgb; T *= e^-tau; stop once 1 - T >= ert.
 *   Output (C, 1 - T) at depth t_in; a miss writes (0,0,0,0) at +inf.
 * Segments whose sample point lies in a macrocell of majorant 0 are skipped;
 * they contribute exactly nothing, so skipping never changes a result.
 * The frame must match the camera's size.  The brick's screen tiles go through
 * the persistent kernel of dpr_render_batch (graph-replayed unless
 * DPR_FLAG_NO_GRAPH); with DPR_FLAG_PLAIN in the render parameters, or with a
 * sample-count buffer attached to `out` (dpr_frame_attach_counts), one plain
 * launch of one thread per pixel renders it instead.  Both give the same bits. */
dpr_status dpr_render_partial(dpr_world, int32_t brick_id, dpr_frame out);

/* Sort-last composite (section 2.1; section 5.1.1): for each pixel, the k
 * fragments with finite depth are sorted by (depth, frag_id) and composited
 * front to back, C += T rgb_i, T *= (1 - alpha_i); output (C, 1 - T) at the
 * minimum depth.  frag_ids are intrinsic ids (e.g. brick or rank), so the
 * result does not depend on the order of `parts`; they must be distinct.
 * 1 <= k <= 256; all frames and `out` have the same size; `out` may not alias
 * a part.  frag_ids may be NULL (ids 0..k-1).                                   */
dpr_status dpr_composite(dpr_device, const dpr_frame* parts, const int32_t* frag_ids, int32_t k,
                         dpr_frame out);

/* dpr_composite for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, hosts that forbid allocation after set-up.
 * Same arguments, same kernels and the same bits as dpr_composite, but every
 * piece of device scratch (fragment table, depth prior, fix-up counters and
 * pixel list) lives in one fixed array of the library, about 33 MB per GPU, held
 * from the first dpr_device_create on that GPU until the process ends.  The call
 * allocates nothing (no hipMalloc/hipFree, no pinned or pageable staging, no
 * host heap on success) and copies nothing from the host: the fragment table
 * travels in kernel arguments.  Limit: out->w * out->h <= 8388608 pixels
 * (3840 x 2160 fits); larger frames return DPR_ERR_UNSUPPORTED.  Every call on
 * one GPU shares that GPU's array: calls enqueued on the same stream are
 * ordered, calls that overlap on different streams of one GPU race (the caller
 * serialises them).  The array keeps the last call's contents; the counters that
 * must start at zero are cleared on the device stream by every call.           */
dpr_status dpr_composite_noalloc(dpr_device, const dpr_frame* parts, const int32_t* frag_ids, int32_t k,
                                 dpr_frame out);

/* The collective render of section 3.2 on one GPU: render every brick of the
 * world to fragments and composite them into `out`.  By default the bricks go
 * through the persistent batched renderer below (one camera); with
 * DPR_FLAG_PLAIN in the render parameters each brick is rendered into its own
 * partial frame by dpr_render_partial and the frames go through dpr_composite.
 * Both give the same bits.                                                      */
dpr_status dpr_render_frame(dpr_world, dpr_frame out);

/* Batched render of n cameras: one persistent launch walks a queue of
 * (camera, brick, screen tile) items, then a tile compositor merges each
 * camera's fragments into outs[c]; replayed from a HIP graph captured on the
 * first call for these frames (flags: DPR_FLAG_PLAIN, DPR_FLAG_NO_GRAPH).
 * The results equal dpr_render_frame per camera bit for bit.                   */
dpr_status dpr_render_batch(dpr_world, const dpr_camera* cams, int32_t n, dpr_frame* outs, uint32_t flags);
/* Time the candidate tile shapes for this world and camera batch on the GPU and
 * keep the fastest for later dpr_render_batch calls; writes the chosen shape.
 * When the environment variable DPR_TUNE_CACHE names a file, the choice is
 * looked up there first (no timing) and stored there after timing, keyed by the
 * device (architecture, CU count) and the shape of the work: voxel type and
 * layout, each brick's stored extent, each camera's image size, step, ERT
 * threshold and macrocell edge (not the camera poses).                          */
dpr_status dpr_autotune_batch(dpr_world, const dpr_camera* cams, int32_t n, dpr_frame* outs,
                              int32_t* tile_w, int32_t* tile_h);
/* Force a tile shape (tile_w * tile_h must be a multiple of 64, <= 1024).      */
/* The tile-shape cache of dpr_autotune_batch (host only, needs no GPU): a JSON
 * object {"version": 1, "entries": {"<key>": [tile_w, tile_h], ...}} in the file
 * `path`.  lookup sets *found to 1 and writes the shape when `key` is there, else
 * *found = 0 (also for a missing or unreadable file).  store adds or replaces
 * the entry, keeping the others, and rewrites the file whole (through a
 * temporary file renamed over it); an unreadable file is replaced.  Keys hold no
 * quote or backslash (DPR_ERR_INVALID_ARGUMENT).                                 */
dpr_status dpr_tune_cache_lookup(const char* path, const char* key, int32_t* found, int32_t* tile_w, int32_t* tile_h);
dpr_status dpr_tune_cache_store(const char* path, const char* key, int32_t tile_w, int32_t tile_h);
dpr_status dpr_set_batch_tile(dpr_world, int32_t tile_w, int32_t tile_h);
/* Durations of the march kernel and of the tile compositor of the last batched
 * render (dpr_render_batch with DPR_FLAG_NO_GRAPH, or dpr_render_frame or
 * dpr_render_partial with DPR_FLAG_NO_GRAPH in the render parameters), from HIP
 * events recorded on the device stream around each kernel.  Synchronises.
 * DPR_ERR_INVALID_STATE when the last batched render was a graph replay (or
 * there was none).                                                              */
dpr_status dpr_batch_timings(dpr_world, float* march_ms, float* composite_ms);

/* Queue coverage of the last batched render, which must have run with
 * DPR_FLAG_QUEUE_COVERAGE (else DPR_ERR_INVALID_STATE): out[0] = queue items
 * ((camera, brick, screen tile) triples), out[1] = items taken exactly once,
 * out[2] = fragment slots (items x tile pixels), out[3] = slots written exactly
 * once.  A complete render has out[1] == out[0] and out[3] == out[2].
 * Synchronises.                                                                 */
dpr_status dpr_batch_coverage(dpr_world, int64_t out[4]);

/* ---------------------------------------------------------------- measurement */
/* Gather ceiling of the local render (a roofline probe, not part of the
 * paradigm): for every pixel of the world's camera, issue the voxel loads that
 * dpr_render_partial makes for brick `brick_id` over the first counts[p] logical
 * samples of the pixel's ray (the same lattice points, the same macrocell skip
 * rule, the same 8-voxel footprints), with no transfer function, no compositing
 * and no dependence between consecutive samples (each ray's samples are cut
 * into slices that separate threads load).  counts (int32) and sink (float; a
 * checksum of the loaded values is added to each pixel's entry) are device
 * arrays of width * height elements, row-major, typically the sample counts a render with a count buffer
 * attached wrote (dpr_frame_attach_counts).  Enqueued on the device stream; the
 * caller times it.                                                              */
dpr_status dpr_measure_gather(dpr_world, int32_t brick_id, const int32_t* counts, float* sink);

/* ---------------------------------------------------------------- deep frames */
/* Section 5.1.1 lets a rank emit possibly several RGBA-z fragments per pixel;
 * section 2.1 (and the interleaved partition of Fig. 6) shows why one is not
 * enough once a rank's data is not convex.  A deep frame holds, per pixel, a
 * fragment count (int32) and up to `capacity` layers of premultiplied RGBA
 * (float4), depth (float) and an intrinsic fragment id (int32), all layer-major:
 * layer i of pixel p sits at index i * w * h + p.  A pixel's fragments occupy
 * layers 0 .. count-1 in front-to-back (depth, id) order; later layers hold
 * unspecified values.  The frame also records the rank that rendered it.
 * 1 <= capacity <= 255.                                                        */
typedef struct dpr_deep_frame_t* dpr_deep_frame;
dpr_status dpr_deep_frame_create(dpr_device, int32_t w, int32_t h, int32_t capacity, dpr_deep_frame* out);
/* Borrow caller device buffers: counts (w*h int32), rgba (capacity*w*h*4 float),
 * depth (capacity*w*h float), ids (capacity*w*h int32); they must outlive the
 * frame.                                                                       */
dpr_status dpr_deep_frame_wrap(dpr_device, int32_t w, int32_t h, int32_t capacity, int32_t* counts, float* rgba,
                               float* depth, int32_t* ids, dpr_deep_frame* out);
void dpr_deep_frame_release(dpr_deep_frame);
/* Render every brick of the world for its camera into a deep frame: per pixel one
 * fragment per brick the ray hits (the fragment dpr_render_partial gives), id =
 * rank * 65536 + brick index, sorted by (depth, id).  The world's bricks may form
 * any non-convex set.  0 <= rank < 32768; the frame's size is the camera's and
 * its capacity is at least the world's brick count, so no pixel can overflow.
 * Runs the batched renderer's march, then a per-tile pass that writes each
 * pixel's sorted fragment list (enqueued directly, or replayed from a HIP graph
 * as dpr_render_batch does; DPR_FLAG_NO_GRAPH in the render parameters).       */
dpr_status dpr_render_deep(dpr_world, int32_t rank, dpr_deep_frame out);
/* Merge k deep frames per pixel and composite front to back into `out`, with the
 * "over" of dpr_composite; depth = the nearest fragment's.  Every live fragment
 * (layer < count) is ranked by (depth, rank of its part, layer), which for frames
 * of dpr_render_deep is their (depth, id) order.  The parts come from distinct
 * ranks (dpr_render_deep), have out's size, and 1 <= k <= 256.  A pixel with n
 * live fragments reads its depths ceil(n / 8) times.  The result does not depend
 * on the order of `parts`.                                                     */
dpr_status dpr_composite_deep(dpr_device, const dpr_deep_frame* parts, int32_t k, dpr_frame out);

/* ---------------------------------------------------------------- path tracing */
/* Data-parallel volumetric path tracing with ray forwarding.  The paper motivates
 * illumination that needs rays to visit content on other ranks (section 2.2;
 * Fig. 7, volumetric shadows) and a path tracer that forwards each ray to the
 * rank holding the content it meets next, so every ray finds its true
 * interactions wherever it was spawned (section 5.2; the wave-front exchange of
 * section 2.2).  Here each brick plays one rank's part: rays advance in waves,
 * and a ray whose next tentative collision lies in another brick is handed to
 * that brick for the next wave.
 * Estimator: extinction D * A(v) (the TF opacity), single-scattering albedo =
 * the TF's RGB, isotropic phase; delta tracking under a piecewise-constant
 * majorant on the global grid of 16^3-cell blocks (D times the TF majorant of
 * the block's value range, walked with a 3D DDA; the grid is global, so the
 * image does not depend on the bricking);
 * at each real collision a shadow ray towards the light estimates the
 * transmittance by ratio tracking and adds thr * light * T / (4 pi); a path
 * leaving the volume box adds thr * env; a path ends after max_bounces real
 * collisions.  Random numbers: Philox4x32-10 (Salmon et al., SC 2011) with key
 * (seed, 0x243F6A88) and counter (path id, event, 0 for the path / 1 for its
 * shadow ray, step), uniform ((x >> 9) + 1/2) 2^-23; path id =
 * (row * width + column) * spp + sample.  Camera rays pass through pixel
 * centres, and a camera path starts in the brick of its first tentative
 * collision (no hand-over counted).  Gaps between bricks are empty space.       */
typedef struct {
  float light_dir[3];    /* direction the light travels (any length > 0)          */
  float light_rgb[3];    /* radiance of the directional light, >= 0                */
  float env_rgb[3];      /* environment radiance seen by paths leaving the box     */
  int32_t max_bounces;   /* real collisions per path, in [1, 255]                  */
  int32_t spp;           /* paths per pixel, >= 1                                  */
  uint32_t seed;         /* first key word of the generator                        */
} dpr_path_params;
typedef struct {
  int64_t paths;         /* camera paths traced                                    */
  int64_t events;        /* tentative collisions of paths (real and null)          */
  int64_t shadow_steps;  /* ratio-tracking steps of shadow rays                    */
  int64_t forwards;      /* hand-overs of a ray to another brick                   */
  int32_t waves;         /* waves until no ray was left                            */
} dpr_path_stats;
/* Render the world's camera into `out`: RGB = mean radiance of the pixel's spp
 * paths, A = 1, depth = +inf.  out's size is the camera's.  Needs a committed
 * world with TF and camera and one element type for all bricks.  Device memory:
 * two ray pools of 64 B x paths x (max_bounces + 1) and 16 B x paths x
 * (max_bounces + 1) of contributions, kept by the world for later calls.
 * Synchronises (the host reads the pool size every few waves).  Of the render
 * flags only DPR_FLAG_WIDE_OFFSETS applies (64-bit voxel offsets on every brick;
 * the same image).  stats may be NULL.                                          */
dpr_status dpr_render_path(dpr_world, const dpr_path_params* params, dpr_frame out, dpr_path_stats* stats);

/* ---------------------------------------------------------------- training */
/* Differentiable render of one whole volume (no bricks, ERT off) for n cameras.
 * volume: FP32 device grid of dims (x fastest); tf: n_tf RGBA FP32 (device).
 * out_rgba (n*H*W*4) / out_depth (n*H*W) are device buffers; `workspace`
 * (device, ws_bytes >= dpr_train_workspace_size) receives, per ray, the total
 * optical depth and a checkpoint every 64 segments, read by the backward pass.  */
dpr_status dpr_train_workspace_size(const int64_t dims[3], const dpr_camera* cams, int32_t n, float step_voxels,
                                    size_t* bytes);
dpr_status dpr_render_train_forward(dpr_device, const float* volume, const int64_t dims[3], const float* tf,
                                    int32_t n_tf, float value_lo, float value_hi, float density,
                                    const dpr_render_params*, const dpr_camera* cams, int32_t n,
                                    float* out_rgba, float* out_depth, void* workspace, size_t ws_bytes);
/* Adjoint: given dL/d(out_rgba) (device, n*H*W*4), ACCUMULATE (+=) dL/dvolume
 * and dL/dtf into the device buffers grad_volume / grad_tf.  Reverse traversal
 * per ray: transmittance is recomputed from the stored total optical depth by
 * subtracting segment depths, restored exactly at every checkpoint.            */
dpr_status dpr_render_backward(dpr_device, const float* volume, const int64_t dims[3], const float* tf,
                               int32_t n_tf, float value_lo, float value_hi, float density,
                               const dpr_render_params*, const dpr_camera* cams, int32_t n,
                               const float* grad_rgba, const void* workspace, size_t ws_bytes,
                               float* grad_volume, float* grad_tf);

#ifdef __cplusplus
}
#endif
#endif /* DPR_H */
