/*
 * scsurf: online surface correction on a voxel-hashed TSDF, for one MI355X
 * (gfx950).  C ABI of the data-parallel hot path of
 *   R. Maier, R. Schaller, D. Cremers, "Efficient Online Surface Correction
 *   for Real-time Large-Scale 3D Reconstruction", arXiv 1709.03763.
 *
 * Every call enqueues its device work on the caller's HIP stream (`stream`,
 * a hipStream_t passed as void*; NULL means the null stream) and returns
 * without synchronising unless stated.  Buffers marked "device" must be
 * device memory that stays valid until the stream has passed the call;
 * buffers marked "host" are read or written before the call returns.  The
 * caller owns every buffer it passes; the library owns the volume (hash
 * table, block pool, counters, scratch, captured graphs).  One volume must
 * not be used from two streams at once.
 *
 * Errors: argument errors are returned at once with nothing enqueued.
 * Errors found on the device (a full hash table or pool, de-integration of
 * an unallocated block, a weight leaving [0, 2^14)) set a sticky error word
 * in the volume, read by sc_volume_query; after such an error the field is
 * unspecified and the volume must be reset and rebuilt by re-integrating the
 * stored keyframes.  No C++ exception crosses this interface.
 *
 * Geometry (Sec. 3, "Preliminaries"): a pose T = (R, t) maps camera to world
 * coordinates, g(T, p) = R p + t, with R row-major.  Cameras are pinhole,
 * u = fx X / Z + cx, v = fy Y / Z + cy, pixel centres at integer
 * coordinates, OpenCV axes (x right, y down, z forward).  Depth is z-depth
 * in metres; 0 marks an invalid pixel.
 *
 * Decision convention (shared by this library and its test oracle, written
 * independently by each): voxel n in Z^3 has centre s*n, block b = floor(n/8)
 * holds 8x8x8 voxels indexed x + 8y + 64z.  Its camera point is the block
 * origin mapped to the camera in FP64 and rounded to FP32, plus the in-block
 * offset added in FP32 along x, then y, then z with per-axis steps
 * fl32(s * R[axis][row]).  The nearest pixel is floor(fl32(fl32(fx*X)/Z)+cx
 * + 1/2) (FP32, correctly rounded, no contraction).  The voxel is touched by
 * a keyframe at a pose iff Z > 0, the pixel is inside the image, the
 * keyframe weight q(W*) = rint(W* 2^10) / 2^10 at the pixel is positive, and
 * |fl32(Z*(pixel) - Z)| <= trunc.
 */
#ifndef SCSURF_H
#define SCSURF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sc_status;
#define SC_OK 0
#define SC_EINVAL (-1)     /* bad argument; nothing enqueued */
#define SC_ENOMEM (-2)     /* a device or host allocation failed */
#define SC_EHASHFULL (-3)  /* sticky: no free bucket in the block hash table */
#define SC_EPOOLFULL (-4)  /* sticky: block pool exhausted (max_blocks) */
#define SC_ENOTALLOC (-5)  /* sticky: de-integration touched an unallocated block */
#define SC_EWEIGHT (-6)    /* sticky: a voxel weight would leave [0, 2^14) */
#define SC_EDEVICE (-7)    /* a HIP runtime call failed */
#define SC_ENOLIB (-8)     /* no usable gfx950 device */
#define SC_ERANGE (-9)     /* sticky: a keyframe pixel's frustum cell spans more than 16 blocks per axis */
#define SC_ESCRATCH (-10)  /* the input needs more than the fixed scratch of an allocation-free entry point */

#define SC_COLOR_RGBA8 0 /* voxel colour 4 x uint8 (RGB + pad); keyframe colour uint8 H x W x 4 */
#define SC_COLOR_F32 1   /* keyframe colour float H x W x 3 in [0,1]; voxel colour held as 3 x double
                            (de-integration amplifies the stored colour's rounding by W / W') */

#define SC_SEL_EQ3 0         /* Eq. (3): the m most-moved consecutive keyframes, ascending index */
#define SC_SEL_TOPM 1        /* the m most-moved keyframes, descending pose change */
#define SC_SEL_ALL_ORDERED 2 /* every changed keyframe, descending pose change */

/* Pinhole intrinsics (Sec. 3); width x height pixels. */
typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;
} sc_intrinsics;

/* Camera-to-world pose (Sec. 3): x_world = R x_cam + t, R row-major. */
typedef struct {
    double R[9];
    double t[3];
} sc_pose;

/* Voxel-hashed SDF (Sec. 3, "SDF volume"). */
typedef struct {
    float voxel_size;      /* metres */
    float trunc;           /* truncation band mu, metres */
    int64_t n_buckets;     /* hash buckets, a power of two */
    int64_t max_blocks;    /* block pool capacity (8^3 voxels each) */
    int32_t color_mode;    /* SC_COLOR_RGBA8 or SC_COLOR_F32 */
    int32_t max_batch_ops; /* capacity of one batched update, in keyframe operations (<= 4096) */
} sc_volume_params;

/* A fused keyframe (Sec. 4.1): depth Z*, fusion weight W*, colour C*.
 * `packed` is optional (NULL: not used): a device copy of the same keyframe
 * interleaved for the voxel passes, H x W records of 16 bytes
 * {float depth', float q(weight), uint32 RGBA8 colour, uint32 0} with
 * q(w) = rint(w 2^10) / 2^10 and depth' = depth where q(weight) > 0, -inf
 * elsewhere (so the band test alone rejects a pixel without weight),
 * followed by the depth range of every 4 x 4 pixel cell:
 * ceil(H/4) x ceil(W/4) pairs {float zmin, float zmax} (row-major) over the
 * cell's valid pixels (q(weight) > 0 and 0 < depth < 1e30), {+inf, -inf}
 * for a cell without one.  16-byte aligned, sc_keyframe_pack_bytes(W, H)
 * bytes, as written by sc_keyframe_pack.  Volumes in RGBA8 mode then read
 * every keyframe sample from it (one gather per voxel instead of three) and
 * the batched candidate stage reads the cell ranges instead of the pixels;
 * FP32-colour volumes ignore it.  It must hold the packing of this
 * keyframe's depth, weight and colour, and is owned by the caller. */
typedef struct {
    const float* depth;  /* device, H x W, metres */
    const float* weight; /* device, H x W; quantised to 2^-10 when used */
    const void* color;   /* device, per the volume's colour mode */
    const void* packed;  /* device, optional, see above */
} sc_keyframe;

/* Keyframe fusion parameters (Sec. 3, "Keyframe Fusion").  kf_fuse and
 * kf_fuse_noalloc require 2^-5 <= z_min <= z_max < 1e6 and non-negative
 * ratios (SC_EINVAL otherwise): the bound on z_min bounds the depth weight
 * 1 / Z^2, which the colour weights are held against in 32 bits. */
typedef struct {
    float z_min, z_max; /* valid depth range, metres */
    float disc_rel;     /* reject a pixel whose 4-neighbour depth differs by more than disc_rel * Z */
    float occ_rel;      /* a colour observation is visible if |Z_i - z| <= occ_rel * z */
} sc_fuse_params;

typedef struct sc_volume sc_volume;

/* Bytes of the packed copy of a width x height keyframe (records and cell
 * depth ranges, see sc_keyframe); 0 for a size outside 1 .. 16384. */
int64_t sc_keyframe_pack_bytes(int32_t width, int32_t height);

/* Writes the packed copy of an RGBA8 keyframe used by the batched passes:
 * packed[i] = {q(weight[i]) > 0 ? depth[i] : -inf, q(weight[i]), color[i], 0}
 * for the width * height pixels (q as in sc_keyframe), then the cell depth
 * ranges.  `packed` is a caller-owned device buffer of `packed_bytes` >=
 * sc_keyframe_pack_bytes(width, height) bytes, 16-byte aligned.  SC_EINVAL
 * on a null pointer, a misaligned or short buffer or a size outside
 * 1 .. 16384; asynchronous on `stream`. */
sc_status sc_keyframe_pack(const sc_keyframe* kf, int32_t width, int32_t height, void* packed, int64_t packed_bytes,
                           void* stream);

/* ---- volume lifecycle --------------------------------------------------- */

/* Creates an empty volume on the current device.  The block pool
 * (max_blocks x 8 KiB in RGBA8 mode, 18 KiB in F32 mode: D in FP64, W in FP32,
 * colour as RGBA8 or 3 x FP64) and the hash table
 * are allocated and cleared here.  *out is NULL on failure. */
sc_status sc_volume_create(const sc_volume_params* params, sc_volume** out);

/* Frees every device and host resource of the volume (synchronises). */
void sc_volume_destroy(sc_volume* vol);

/* Empties the volume (all blocks freed, error word cleared); enqueued. */
sc_status sc_volume_reset(sc_volume* vol, void* stream);

/* Synchronises `stream` and returns the allocated block count and the sticky
 * device error (SC_OK or one of the sticky codes above). */
sc_status sc_volume_query(sc_volume* vol, void* stream, int64_t* n_blocks, int32_t* sticky_error);

/* Copies the first min(n_blocks, cap) allocated blocks, in pool order, into
 * device buffers: block coordinates (int32 x 3), D (float x 512, rounded
 * to nearest from the FP64 voxel value), W (float x
 * 512) and colour (uint32 RGBA8 x 512, or float x 3 x 512 planar, rounded
 * from the FP64 voxel colour).  Any
 * output may be NULL.  *n_out (host) receives n_blocks.  Synchronises. */
sc_status sc_volume_export(sc_volume* vol, void* stream, int32_t* block_xyz, float* D, float* W, void* C,
                           int64_t cap, int64_t* n_out);

/* Loads blocks into the volume (the inverse of sc_volume_export, for
 * checkpoints and for meshing given fields): block coordinates (device int32
 * n x 3) are allocated as by hash_alloc and each block's record is written
 * from D (device float n x 512, stored in FP64), W (float n x 512; weights
 * belong on the 2^-10 grid below 2^14, not checked) and C (uint32 RGBA8
 * n x 512, or float n x 3 x 512 planar in FP32-colour mode), in the layout
 * sc_volume_export writes; a NULL field is stored as zeros.  Blocks already
 * present are overwritten; with duplicate coordinates in one call, which
 * record lands is unspecified.  SC_EINVAL if n exceeds max_blocks;
 * synchronises and returns the sticky error (SC_EPOOLFULL, SC_EHASHFULL). */
sc_status sc_volume_import(sc_volume* vol, void* stream, const int32_t* block_xyz, const float* D, const float* W,
                           const void* C, int64_t n);

/* ---- keyframe fusion (Sec. 3 "Keyframe Fusion", Eq. 1) ------------------- */

/* Overlap of a frame with a keyframe's reference view (Sec. 4.2, the
 * overlap strategy for starting a new keyframe).  A pixel of `depth` is
 * valid if z_min <= Z <= z_max; it is visible if its back-projected point,
 * moved into the reference camera (T_ref^-1 T_frame), lies in front of it
 * and its nearest pixel there is inside the image.  Computed in FP64 in the
 * written order (camera point ((u - cx) / fx) Z, ((v - cy) / fy) Z, Z; world
 * point R p + t row by row; reference point R_ref^T (w - t_ref) column by
 * column; pixel floor(fx x / z + cx + 1/2)).  counts: device, 2 x uint32
 * {valid, visible}, overwritten.  depth: device H x W.  SC_EINVAL on a null
 * pointer or bad intrinsics; asynchronous on `stream`. */
sc_status sc_overlap(const float* depth, const sc_intrinsics* intr, const sc_pose* T_frame, const sc_pose* T_ref,
                     float z_min, float z_max, uint32_t* counts, void* stream);

/* Per-pixel depth weight w_z = cos(theta) Z^-2, theta the angle between the
 * depth normal and the camera axis, quantised to 2^-10; 0 marks pixels that
 * are invalid or near a depth discontinuity.  depth: device n x H x W;
 * wz_out: device n x H x W. */
sc_status sc_depth_weight(const float* depth, int32_t n_frames, const sc_intrinsics* intr,
                          const sc_fuse_params* params, float* wz_out, void* stream);

/* Colour pre-processing of n frames: unsharp masking with the binomial
 * [1 4 6 4 1]/16 kernel (amount 1), exact, in units of 1/256 (device uint16
 * n x H x W x 3), and the blurriness weight w_b = 1 - blur of each frame
 * (device double n), blur the re-blur measure of Crete et al. (2007). */
sc_status sc_color_prep(const uint8_t* rgb, int32_t n_frames, int32_t width, int32_t height, uint16_t* sharp_out,
                        double* wb_out, void* stream);

/* Fuses n consecutive frames into one keyframe with pose T* = poses[ref]:
 * forward-warped weighted depth average (Eq. 1) and weighted-median colour of
 * the back-warped, sharpened input colours with weights w_b * w_z.  depth:
 * device n x H x W float; rgb: device n x H x W x 3 uint8; poses: host n.
 * Outputs (device, H x W): kf_depth, kf_weight (on the 2^-10 grid), kf_rgba
 * (uint8 x 4, alpha 255 on valid pixels).  n_frames <= 64.  Scratch is held
 * by the library between calls and reused (one set per device), so calls
 * that overlap on one device (two streams) race and must be ordered by the
 * caller.  Relative poses travel as kernel arguments: the host does not wait
 * for the device. */
sc_status kf_fuse(const float* depth, const uint8_t* rgb, const sc_pose* poses, int32_t n_frames, int32_t ref,
                  const sc_intrinsics* intr, const sc_fuse_params* params, float* kf_depth, float* kf_weight,
                  uint8_t* kf_rgba, void* stream);

/* kf_fuse for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same arguments,
 * kernels and results, with every intermediate buffer (per-frame weights,
 * sharpened colour, fixed-point accumulators, colour-prep partials, relative
 * poses) in one fixed 76 MiB device array per device, held until the process
 * ends.  Relative poses travel as kernel arguments, so no host staging or
 * copy is enqueued either.  The array needs about
 * 16 H W + 12 H W n_frames bytes (640 x 480 fits up to 20 frames); a larger
 * input returns SC_ESCRATCH with nothing enqueued.  Every call on a device
 * shares that device's array, so calls that overlap on one device (two
 * streams, or two host threads) race and must be ordered by the caller.
 * The first call on a device looks up the array's address there. */
sc_status kf_fuse_noalloc(const float* depth, const uint8_t* rgb, const sc_pose* poses, int32_t n_frames,
                          int32_t ref, const sc_intrinsics* intr, const sc_fuse_params* params, float* kf_depth,
                          float* kf_weight, uint8_t* kf_rgba, void* stream);

/* ---- voxel blocks (Sec. 3 "SDF volume") --------------------------------- */

/* Allocates the blocks whose coordinates are listed (device int32 n x 3,
 * duplicates allowed): hash probe and insert, one pool slot per new key.
 * slots_out (device int32 n, may be NULL) receives each entry's pool slot. */
sc_status hash_alloc(sc_volume* vol, const int32_t* block_xyz, int64_t n, int32_t* slots_out, void* stream);

/* Integrates one keyframe at pose T (Sec. 3: blocks are first allocated,
 * then voxels updated with a running weighted average):
 *   W' = W + w, D' = (D W + d w) / W', C' = (C W + c w) / W',
 * d = Z*(pixel) - Z (projective distance along z), w = q(W*(pixel)).  RGBA8
 * colour is rounded to nearest, ties to even, after the update. */
sc_status tsdf_integrate(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* intr, const sc_pose* T,
                         void* stream);

/* Integrates n_kf keyframes at poses T (host, n_kf), in order, each by the
 * running weighted average of Sec. 3 (the update of tsdf_integrate above):
 * the same result, bit for bit, as n_kf tsdf_integrate calls in that order,
 * from the batched path (candidate blocks of all of them at once, then one
 * persistent launch applying each voxel's integrations in order; chunks of
 * the volume's max_batch_ops).  Every keyframe is intr's width x height.
 * SC_EINVAL on a null pointer, n_kf <= 0 or bad intrinsics, with nothing
 * enqueued.  For the pipeline of Sec. 4.1 when several finished keyframes
 * may wait before the volume must show them (until the next pose-graph
 * update).  kfs and T are read during the call; the keyframes' device
 * buffers must stay valid until the work on `stream` completes. */
sc_status tsdf_integrate_batch(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                               const sc_pose* T, void* stream);

/* De-integrates one keyframe at pose T, Eq. (2) (Sec. 4.3):
 *   W' = W - w, D' = (D W - d w) / W', C' = (C W - c w) / W',
 * with W' = 0 giving the empty voxel (0, 0, 0).  Never allocates. */
sc_status tsdf_deintegrate(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* intr, const sc_pose* T,
                           void* stream);

/* ---- surface correction (Sec. 4.3) --------------------------------------- */

/* Host-only selection of keyframes to re-integrate.  Pose change
 * ||s o t_i - s o t_i'||, t the Z-Y-X Euler angles and translation,
 * s = (2,2,2,1,1,1); mode SC_SEL_*.  Writes indices in processing order to
 * `out` (host, >= K) and the distances to dist_out (host, K, may be NULL).
 * Returns the number selected, or a negative status. */
int32_t sc_select(const sc_pose* T, const sc_pose* T_new, int32_t K, int32_t m, int32_t mode, int32_t* out,
                  double* dist_out);

/* The same selection from given distances (host, K). */
int32_t sc_select_dist(const double* dist, int32_t K, int32_t m, int32_t mode, int32_t* out);

/* Motion of a frame pose T relative to a keyframe's first pose T_kf, the
 * quantities of the distance keyframe strategy (Sec. 4.2): *trans = |d| and
 * *angle = atan2(sin, cos) of the rotation of T_kf^-1 T = (A, d), with
 * A - A^T = 2 sin [axis]x and trace A = 1 + 2 cos (radians, [0, pi]).
 * Host only, FP64.  SC_EINVAL on a null pointer. */
sc_status sc_relative_motion(const sc_pose* T_kf, const sc_pose* T, double* trans, double* angle);

/* Applies one pose-graph update in a single batched pass: selects keyframes
 * (mode, m), de-integrates each selected keyframe at its integration pose
 * and re-integrates it at its new pose (all de-integrations first, then all
 * re-integrations, each in processing order; Sec. 4.3), every voxel applying
 * its operations in that order.  One persistent, graph-captured launch does
 * the voxel work.  All keyframes must share width and height.
 * T_integrated (host, n_kf) is updated to T_new for the selected keyframes.
 * selected_out (host, n_kf, may be NULL) receives the processing order and
 * *n_selected (host, may be NULL) its length. */
sc_status reintegrate_batch(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                            sc_pose* T_integrated, const sc_pose* T_new, int32_t m, int32_t mode,
                            int32_t* selected_out, int32_t* n_selected, void* stream);

/* The plain per-keyframe path with the same semantics as reintegrate_batch:
 * one tsdf_deintegrate per selected keyframe, then one tsdf_integrate each. */
sc_status reintegrate_plain(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                            sc_pose* T_integrated, const sc_pose* T_new, int32_t m, int32_t mode,
                            int32_t* selected_out, int32_t* n_selected, void* stream);

/* Schedule of the batched voxel pass.
 *   vpl          voxels per lane: 8, 4, 2 or 1; a block is handled by 8 / vpl
 *                wavefronts.
 *   waves_per_wg wavefronts per workgroup.  Derived (4 for vpl 8, else
 *                8 / vpl) unless `compact` is set, where it may be 1, 2 or 4.
 *   wgs_per_cu   persistent workgroups per compute unit, 1..32.
 *   compact      0: each lane updates its own voxels, block state held in
 *                registers.  1, 2 or 3 (vpl 8 only): block state held in
 *                LDS, the touched voxels of each operation are gathered into
 *                an LDS queue and updated by all 64 lanes together; 2 tests
 *                a lane's voxels four at a time (fewer registers); 3 does as
 *                2 and issues the keyframe gathers of the next four voxels
 *                (or the next operation) before updating the current ones;
 *                4 does as 3 with the touched voxels of an operation
 *                collected in a ring and updated 64 at a time, and the block
 *                geometry computed once per (block, operation).
 * Every schedule gives identical bits.  sc_set_schedule validates and stores
 * it in the volume (SC_EINVAL otherwise); sc_get_schedule reads it back.  A
 * new volume holds {8, 2, 8, 4} (RGBA8 colour) or {8, 4, 4, 0} (FP32
 * colour). */
typedef struct {
    int32_t vpl;
    int32_t waves_per_wg;
    int32_t wgs_per_cu;
    int32_t compact;
} sc_schedule;
sc_status sc_set_schedule(sc_volume* vol, const sc_schedule* sched);
sc_status sc_get_schedule(sc_volume* vol, sc_schedule* sched);

/* Autotuner: times every schedule on a private copy of the volume running the
 * given update (nothing in `vol` changes), stores the fastest in the volume,
 * and writes it to *best (host, may be NULL) with its time in *best_ms.
 * Results are cached for the process, keyed by the GPU architecture, the
 * image size, the operations per chunk, whether the keyframes are packed
 * and the volume parameters; a call whose key is cached sets the cached
 * schedule without timing.  sc_autotune_clear empties the cache. */
sc_status sc_autotune(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                      const sc_pose* T_integrated, const sc_pose* T_new, int32_t m, int32_t mode,
                      sc_schedule* best, float* best_ms, void* stream);
void sc_autotune_clear(void);

/* Measurement of the batched voxel pass: HIP events are recorded on the
 * caller's stream immediately before and after the persistent voxel pass of
 * each of the next `capacity` batched launches (0 disables and frees them).
 * Synchronises the device. */
sc_status sc_batch_timing(sc_volume* vol, int32_t capacity);

/* Elapsed milliseconds of the voxel pass of each recorded launch (host
 * array of at least the capacity); *n (host) receives their number.  Waits
 * for the recorded events. */
sc_status sc_batch_timing_read(sc_volume* vol, float* ms, int32_t* n);

/* Cumulative counters of the batched voxel pass since the volume was
 * created or reset (host int64[4]): candidate blocks processed, (block,
 * operation) pairs tested, touched voxel updates applied, blocks written.
 * Synchronises `stream`. */
sc_status sc_volume_stats(sc_volume* vol, void* stream, int64_t* stats);

/* ---- memory-capped streaming (Sec. 3 "SDF volume", Sec. 4.3) ------------ */

/* Streaming mode: the device pool (max_blocks) holds the blocks near the
 * camera, the others live in a host store.  With enable != 0 every
 * tsdf_integrate, tsdf_deintegrate, reintegrate_batch and reintegrate_plain
 * first streams in, from the host store, exactly those of its candidate
 * blocks the store holds (one synchronisation per operation or batch chunk),
 * so every operation sees every block it may touch and the field equals,
 * bit for bit, the one a resident volume would hold.  A stream-in that does
 * not fit the pool sets the sticky SC_EPOOLFULL; any other failure of the
 * streaming step (SC_ENOMEM, SC_EDEVICE) is made sticky too, since the
 * operation is left undone.  Disabling fails
 * (SC_EINVAL) while the host store holds blocks.  hash_alloc,
 * sc_volume_import and tsdf_integrate_backward return SC_EINVAL while it
 * does; export, mesh and stats see the device blocks only.  The host store
 * is emptied by sc_volume_reset and freed with the volume. */
sc_status sc_stream_enable(sc_volume* vol, int32_t enable);

/* Streams out (to the host store) every device block whose centre
 * s (8 b + 3.5) lies farther than `radius` metres from center (host
 * double[3], world frame) and compacts the pool; the streaming sphere of
 * Sec. 3 around the camera position.  Synchronises `stream`.  SC_EINVAL
 * outside streaming mode or for a negative radius. */
sc_status sc_stream_out(sc_volume* vol, const double* center, double radius, void* stream);

/* Streams every host-held block back in (SC_EPOOLFULL, sticky, if they do
 * not fit).  Synchronises `stream`. */
sc_status sc_stream_in_all(sc_volume* vol, void* stream);

/* The blocks the host store holds, in sc_volume_export's layout but into
 * HOST buffers (any may be NULL): block_xyz int32 n x 3, D and W float
 * n x 512, C uint32 n x 512 (RGBA8) or float n x 3 x 512 (FP32 colour); at
 * most cap blocks are written, *n_out receives their number.  With
 * sc_volume_export it gives the whole field of a streamed volume. */
sc_status sc_stream_export(sc_volume* vol, int32_t* block_xyz, float* D, float* W, void* C, int64_t cap,
                           int64_t* n_out);

/* Host int64[6]: device blocks, host blocks, blocks streamed out and in so
 * far, and the same in bytes.  Synchronises `stream`. */
sc_status sc_stream_stats(sc_volume* vol, void* stream, int64_t* stats);

/* ---- adjoint of integration --------------------------------------------- */

/* Backward of integrating n_kf keyframes at poses T_k Exp(xi_k) (xi at 0)
 * into a field with prior (D0, C0, W0) (Sec. 3 running weighted average;
 * d and w of Sec. 4.3), with the pixel and band decisions of the forward held
 * fixed.  With a = w_k / W(v) per touched (voxel, keyframe) and
 * W0(v) = W(v) - sum_k w_k(v):
 *   dL/dZ_k(u)   += sum_{v -> u} a dL/dD(v)
 *   dL/dC_k(u)   += sum_{v -> u} a dL/dC(v)               (F32 colour only)
 *   dL/dxi_k     += sum_v a dL/dD(v) (0, 0, 1, p_y, -p_x, 0), p = T_k^-1 x_v
 *   dL/dD0(v)     = (W0 / W) dL/dD(v), dL/dC0(v) = (W0 / W) dL/dC(v)
 * (0 where W = 0; W0 is formed exactly on the 2^-10 weight grid before
 * the one division, so a small W0 / W keeps its relative precision).  The
 * volume must hold the field after the forward, with no sticky error
 * (returned as the status otherwise).  grad_D (device,
 * n_blocks x 512) and grad_C (device, n_blocks x 3 x 512, may be NULL) are
 * indexed by pool slot.  Accumulated outputs (callers zero them): grad_depth
 * (device n_kf x H x W), grad_color (device n_kf x H x W x 3; NULL exactly
 * when grad_C is; F32-colour volumes only), grad_xi (device n_kf x 6, FP32).
 * Written outputs (may be NULL; grad_C0 needs grad_D0 and grad_C): grad_D0
 * (device n_blocks x 512), grad_C0 (device n_blocks x 3 x 512), by pool
 * slot.  The keyframes run in chunks of up to min(max_batch_ops, 512)
 * through the batched candidate stage; each candidate block is visited once
 * per chunk.  The order of the FP32 atomic additions into grad_depth and
 * grad_color is not fixed.  SC_EINVAL for a missing required pointer,
 * grad_color on an RGBA8 volume or bad intrinsics. */
sc_status tsdf_integrate_backward(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                                  const sc_pose* T, const float* grad_D, const float* grad_C, float* grad_depth,
                                  float* grad_color, float* grad_xi, float* grad_D0, float* grad_C0, void* stream);

/* ---- iso-surface and surface metrics (Sec. 3; Sec. 5 evaluation) -------- */

/* Marching Cubes over the volume (Sec. 3 "SDF volume": the iso-surface of
 * D = 0 is extracted with Marching Cubes).  The cube of voxel n has corners
 * n + {0,1}^3 and is meshed only when all eight corner voxels are allocated
 * with W > 0; a corner is inside when D < 0.  The vertex on a crossing edge
 * from voxel p to p + e_a is s (p + t e_a), t = D(p) / (D(p) - D(p + e_a)),
 * in FP64 from the FP64 voxel D, rounded to FP32.  Triangulation: on each
 * cube face the runs of inside corners are cut off one by one (diagonal
 * inside corners stay apart), the face segments chain into loops, a loop is
 * fanned from its smallest edge, or from an added centre vertex (the mean of
 * its vertices) when it crosses one face twice; triangles face increasing D,
 * and the mesh is closed wherever all cubes around it are meshed.
 * Outputs (device, may be NULL): tri_xyz cap x 3 x 3 FP32 vertex positions
 * (metres, world frame), tri_keys cap x 3 x 4 int32 vertex keys (x, y, z, k):
 * k < 3 the edge along axis k from voxel (x, y, z), k = 3 + j the centre of
 * loop j in the cube of voxel (x, y, z).  Triangles come in a fixed order
 * (blocks in pool order, cubes in voxel order within a block); the first
 * min(count, cap) are written and *n_tri (host) receives the count, so a
 * call with cap = 0 sizes the buffers.  Allocates temporaries (per-block
 * counts and offsets); synchronises. */
sc_status sc_volume_mesh(sc_volume* vol, void* stream, float* tri_xyz, int32_t* tri_keys, int64_t cap,
                         int64_t* n_tri);

/* The case table sc_volume_mesh uses, as built on the host (no device
 * work): loops (host, 256 x 16 bytes) holds, per case (bit k set = corner k
 * inside), its loops in order, each a header byte (vertex count, | 0x80
 * when fanned around a centre vertex) followed by its edge numbers, ended by
 * a zero header or the 16th byte; ntri (host, 256 bytes) the triangle count
 * per case.  Either may be NULL, not both. */
sc_status sc_mesh_table(uint8_t* loops, uint8_t* ntri);

/* The mesh's vertices, one per key (Sec. 5 measures distances between mesh
 * vertices): tri_xyz / tri_keys as written by sc_volume_mesh (device, n_tri
 * triangles); vert_xyz (device, cap x 3 FP32) receives the first
 * min(count, cap) distinct vertices in no fixed order, *n_vert (host) the
 * count.  SC_ERANGE if a voxel coordinate is outside [-2^19, 2^19).
 * Allocates a temporary hash set; synchronises. */
sc_status sc_mesh_vertices(const float* tri_xyz, const int32_t* tri_keys, int64_t n_tri, float* vert_xyz, int64_t cap,
                           int64_t* n_vert, void* stream);

/* Capped nearest-neighbour distances (Sec. 5 "Surface evaluation methods and
 * metrics": CORR is the mean over the mesh vertices of the distance to the
 * nearest reference point, COMPL the mean over the reference of the distance
 * to the nearest mesh vertex).  For every query point (device, n_query x 3
 * FP32) the Euclidean distance to the nearest point of ref (device, n_ref x
 * 3 FP32), computed in FP32 as sqrt((dx^2 + dy^2) + dz^2), capped at radius
 * (a query with no reference point within the radius, or an empty ref, gets
 * the radius).  dist (device, n_query FP32) may be NULL; sum (device, one
 * FP64) receives the sum of the distances when not NULL.  Exact search over a
 * uniform grid of cells slightly larger than the radius, valid while
 * |coordinate| / radius < 10^5.  SC_EINVAL for a radius that is not positive
 * and finite.  Allocates temporaries; synchronises. */
sc_status sc_nn_distance(const float* ref, int64_t n_ref, const float* query, int64_t n_query, float radius,
                         float* dist, double* sum, void* stream);

/* Library version string. */
const char* sc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCSURF_H */
