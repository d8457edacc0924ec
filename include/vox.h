/*
 * vox.h - C ABI of the MI355X (gfx950) parametric segment voxelizer.
 *
 * The operation (arXiv 2009.09500, Section 3): a segment with start point S
 * and end point E is decomposed into the voxels that contain the points
 *     G_k = S + W k,  W = (E - S) / N,  k = 0, 1, ..., N      (eq. (2)-(3))
 * emitted in order as the array V^(k) (algorithm of Fig. 3).  This library
 * fixes what the paper leaves open:
 *   N            = max(|dx|, |dy|, |dz|)  (Chebyshev length; eq. (1) of the
 *                  paper uses the integer part of the Euclidean length),
 *   k            = 0..N, so a segment has N + 1 voxels and both end points,
 *   voxel of G_k = floor(G_k + 1/2) per axis (centres on integers, ties
 *                  rounded up), evaluated exactly in integers as
 *                  P0_a + floor((2 k d_a + N) / (2 N)),
 *   S == E       gives the single voxel S.
 * Many segments are handled in one call, as the paper's multi-segment
 * experiments do in one kernel call (Section 4 and Section 5, experiment 3).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HBM of the current HIP device),
 *     h_* are host pointers.  The caller allocates and frees all of them,
 *     including the workspace d_work; the library keeps no pointer after a
 *     call returns and allocates no device memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call is stream-ordered and asynchronous unless it says it
 *     synchronises.
 *   - Argument errors detectable on the host are returned at once and launch
 *     nothing.  Errors that depend on device data (end points out of range,
 *     list capacity exceeded) are recorded in the device status word, the
 *     first int32 of d_work, as a vox_status code; vox_read_status() fetches
 *     it.  Such errors never cause an out-of-bounds write: the affected
 *     output is left unwritten, as each entry point states.
 *   - Entry points are re-entrant.  Calls that share a workspace must be
 *     ordered (same stream, or synchronised).  vox_last_error() is
 *     thread-local.
 */
#ifndef VOX_H
#define VOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VOX_ABI_VERSION 4

/* One segment: start point (x0,y0,z0) = S, end point (x1,y1,z1) = E.
 * Arrays of segments are dense, 24 bytes per segment, 4-byte aligned. */
typedef struct vox_segment {
    int32_t x0, y0, z0, x1, y1, z1;
} vox_segment;

typedef enum vox_status {
    VOX_OK = 0,
    VOX_ERR_INVALID_ARGUMENT = 1, /* bad pointer, size or flag            */
    VOX_ERR_OUT_OF_RANGE = 2,     /* an end point outside the output range */
    VOX_ERR_CAPACITY = 3,         /* voxel list larger than the capacity   */
    VOX_ERR_DEVICE = 4,           /* a HIP runtime call failed             */
    VOX_ERR_WORKSPACE = 5,        /* workspace missing or too small        */
    VOX_ERR_BATCH_MISMATCH = 6    /* batch table does not fit its launch   */
} vox_status;

/* Grid flag: zero the whole bit-volume before setting voxels.  Without it
 * the voxels are ORed into the volume's current contents. */
#define VOX_GRID_CLEAR 1u
/* Grid flag: the paper's literal length of eq. (1), N = int(|E - S|) (see
 * vox_segments_to_list_euclid), instead of max |d_a|.  Such calls take the
 * direct path (one device atomic per voxel, no LDS bricks). */
#define VOX_GRID_EUCLID 2u

/* ---------------------------------------------------------------- lists */

/* Workspace bytes for vox_segments_to_list with n segments and a voxel
 * buffer of `capacity` voxels (capacity may be 0 for a size query). */
size_t vox_list_workspace_bytes(int64_t n, int64_t capacity);

/* Per-segment voxel lists (Fig. 3, output "array of voxels V^(k)").
 *
 *   d_segs     [n] segments, device.
 *   n          number of segments, >= 0.
 *   d_offsets  [n+1] int64 out, device: d_offsets[i] = sum_{j<i} (N_j + 1),
 *              d_offsets[n] = total voxel count.  Always written.
 *   d_voxels   [capacity][3] int16 out, device: voxel k of segment i is row
 *              d_offsets[i] + k, columns x,y,z; segments in input order,
 *              voxels from S to E.  NULL = size query (offsets only).
 *   capacity   rows available in d_voxels (>= 0).
 *   h_total    optional host out.  If non-NULL the call synchronises the
 *              stream once, stores the total, and returns
 *              VOX_ERR_OUT_OF_RANGE / VOX_ERR_CAPACITY from the device
 *              status instead of VOX_OK.
 *   d_work     workspace, >= vox_list_workspace_bytes(n, capacity) bytes,
 *              256-byte aligned.
 *
 * Device-checked: every coordinate must lie in [-32768, 32767] (int16
 * output) and total <= capacity; otherwise the status word is set and no
 * voxel row is written (offsets still are). */
vox_status vox_segments_to_list(const vox_segment *d_segs, int64_t n,
                                int64_t *d_offsets, int16_t *d_voxels,
                                int64_t capacity, int64_t *h_total,
                                void *d_work, size_t work_bytes, void *stream);

/* The same lists with the paper's literal length of eq. (1): N_i =
 * int(|E - S|) (the integer square root of dx^2 + dy^2 + dz^2), samples
 * S + k (E - S) / N_i for k = 0..N_i (eq. (2)-(3)) each mapped to the voxel
 * containing it (round half up, as above), and a sample that falls in the
 * voxel of the sample before it dropped (with this N two samples can share
 * a voxel).  d_offsets[i] counts the voxels kept; arguments, workspace size
 * (vox_list_workspace_bytes), ownership and errors as for
 * vox_segments_to_list.  Sixteen lanes share a segment's samples. */
vox_status vox_segments_to_list_euclid(const vox_segment *d_segs, int64_t n,
                                       int64_t *d_offsets, int16_t *d_voxels,
                                       int64_t capacity, int64_t *h_total,
                                       void *d_work, size_t work_bytes, void *stream);

/* The same lists as vox_segments_to_list with int32 coordinates, for
 * segments whose voxels leave the int16 range (Section 5 times single
 * segments of up to 10^6 voxels).  d_voxels is [capacity][3] int32, 16-byte
 * aligned; every other argument, the workspace size
 * (vox_list_workspace_bytes), ownership and the errors are those of
 * vox_segments_to_list, except the range rule: every axis difference
 * |P1_a - P0_a| must be below 2^30 (any int32 end points otherwise), else
 * VOX_ERR_OUT_OF_RANGE (with h_total) and no voxel row is written. */
vox_status vox_segments_to_list32(const vox_segment *d_segs, int64_t n,
                                  int64_t *d_offsets, int32_t *d_voxels,
                                  int64_t capacity, int64_t *h_total,
                                  void *d_work, size_t work_bytes, void *stream);

/* ----------------------------------------------------------------- grids */

/* Workspace bytes for vox_segments_to_grid with n segments and the given
 * volume (the bound covers the worst case of every segment crossing the
 * whole volume). */
size_t vox_grid_workspace_bytes(int64_t n, int32_t dim_x, int32_t dim_y, int32_t dim_z);

/* Packed occupancy bit-volume of all voxels of all segments (the "scene
 * voxel array" that the generated primitives are assembled into, Section 2
 * and Section 3 around Fig. 1).
 *
 *   dim_x, dim_y, dim_z  volume size in voxels, each in [1, 2^20] and
 *              dim_x*dim_y*dim_z <= 2^38.
 *   d_grid     [ceil(dim_x*dim_y*dim_z / 32)] uint32, device, in/out.
 *              Voxel (x,y,z) is bit b = (z*dim_y + y)*dim_x + x, stored in
 *              word b / 32 at bit b % 32 (least significant bit first).
 *   d_counts   optional [n] int32 out, device: N_i + 1 (with
 *              VOX_GRID_EUCLID: the voxels kept, 0 for a segment outside the
 *              volume).
 *   flags      VOX_GRID_CLEAR and/or VOX_GRID_EUCLID, or 0.
 *   d_work     workspace, >= vox_grid_workspace_bytes(...) bytes, 256-byte
 *              aligned.
 *
 * Device-checked: both end points of a segment must lie inside the volume
 * (then every voxel does, as each coordinate is rounded from a value between
 * two in-range integers).  A segment that fails sets VOX_ERR_OUT_OF_RANGE
 * and contributes no voxel; the others are still written.
 *
 * Calls with more than 16384 segments, 8-byte-aligned d_segs, the
 * Chebyshev N, dim_x a multiple of 32 and every side at most 16384 (and a
 * brick count within the library's limit) fill LDS bricks; the others take
 * the direct path (one device atomic per voxel).  The output is the same. */
vox_status vox_segments_to_grid(const vox_segment *d_segs, int64_t n,
                                int32_t dim_x, int32_t dim_y, int32_t dim_z,
                                uint32_t *d_grid, int32_t *d_counts, uint32_t flags,
                                void *d_work, size_t work_bytes, void *stream);

/* ----------------------------------------------------------------- tuning */

/* Launch-shape choice for bit-volume calls.  brick_lg[a] is log2 of the LDS
 * brick size along axis a; all zero selects the library default.  The
 * choice changes only speed and workspace size, never the output.  Supported
 * shapes: 2^8 x 2^6 x 2^5, 2^8 x 2^6 x 2^6, 2^7 x 2^6 x 2^6, 2^7 x 2^7 x 2^6. */
typedef struct vox_tuning {
    int32_t brick_lg[3];
} vox_tuning;

/* Sets the process-wide tuning used by later grid and batch calls (NULL
 * restores the default).  Workspace sizes depend on it: query them after
 * setting it.  VOX_ERR_INVALID_ARGUMENT for an unsupported shape. */
vox_status vox_set_tuning(const vox_tuning *tuning);

/* Current process-wide tuning. */
vox_status vox_get_tuning(vox_tuning *tuning);

/* ---------------------------------------------------------------- batches */

/* One scene of a batch: its own segments and its own bit-volume, with the
 * meaning of the vox_segments_to_grid arguments of the same names.  Batch
 * scenes take the brick path: dim_x must be a multiple of 32 and every
 * side at most 16384, with at most 16384 bricks per scene. */
typedef struct vox_scene {
    const vox_segment *segs; /* device, 8-byte aligned; may be NULL if n == 0 */
    int64_t n;
    int32_t dim_x, dim_y, dim_z;
    uint32_t flags;          /* VOX_GRID_CLEAR or 0 */
    uint32_t *grid;          /* device, 16-byte aligned */
    int32_t *counts;         /* device, optional (NULL) */
} vox_scene;

/* Launch shape of a batch: the kernels are sized by these values, and a
 * table fits a launch when its own values stay within them (same brick
 * shape).  Filled in by vox_batch_plan; vox_batch_launch_cover widens one
 * launch to cover another, so one captured graph can serve several tables. */
typedef struct vox_batch_launch {
    int64_t rows;                 /* histogram workgroups                  */
    int64_t bricks;               /* bricks over all scenes                */
    int32_t brick_lg[3];          /* brick shape (log2 voxels per axis)     */
    int32_t max_scene_bricks;     /* largest per-scene brick count         */
    uint64_t work_bytes;          /* workspace bytes the launch needs      */
    uint64_t table_bytes;         /* bytes of the table image              */
} vox_batch_launch;

/* Host-side planning of a batch (no device call is made).  From the host
 * array h_scenes[n_scenes] (n_scenes >= 1; its pointers are device
 * pointers) build the table image in h_table (host memory, h_table_bytes
 * long) and describe the launch in *launch.  Pass h_table = NULL to fill
 * *launch only (launch->table_bytes is the size to provide).  The brick
 * shape is the process-wide tuning if set, else the default of the largest
 * scene.  The caller copies the image to device memory (any way it likes,
 * 16-byte aligned) before vox_batch_scenes runs; the copy must stay valid
 * until the batch's kernels have finished.
 * Host-checked errors: the vox_segments_to_grid argument rules per scene
 * (VOX_ERR_INVALID_ARGUMENT, with the scene index in vox_last_error), a
 * volume the brick path cannot take, h_table_bytes too small, totals beyond
 * 2^32 - 1 bricks or pieces. */
vox_status vox_batch_plan(const vox_scene *h_scenes, int32_t n_scenes,
                          void *h_table, size_t h_table_bytes,
                          vox_batch_launch *launch);

/* Grows *bound so that every table fitting *launch also fits *bound
 * (element-wise maximum).  VOX_ERR_INVALID_ARGUMENT if the brick shapes
 * differ (a zeroed *bound takes the shape of *launch). */
vox_status vox_batch_launch_cover(vox_batch_launch *bound, const vox_batch_launch *launch);

/* All scenes of a planned batch in one launch sequence of the grid
 * kernels, each kernel a single launch over every scene (the paper's advice
 * to cut the number of kernel calls and load the GPU with many segments at
 * once, Section 5, conclusions), with the bricks of all scenes taken from
 * one work-stealing counter by persistent workgroups.  Every scene's grid
 * (and counts) ends up exactly as a separate vox_segments_to_grid call
 * would leave it; the device status word covers all scenes.
 *
 *   d_table    device copy of a table image from vox_batch_plan.
 *   launch     launch shape (host struct): the plan's own, or a cover of
 *              several plans.
 *   d_work     workspace, >= launch->work_bytes, 256-byte aligned.
 *
 * Reads no device memory on the host, synchronises nothing and allocates
 * nothing, so it can be captured into a HIP graph once and replayed after
 * the caller rewrites d_table (same address) with another table that fits
 * `launch`.  Device-checked: a table that does not fit the launch or the
 * workspace writes nothing and sets VOX_ERR_BATCH_MISMATCH. */
vox_status vox_batch_scenes(const void *d_table, const vox_batch_launch *launch,
                            void *d_work, size_t work_bytes, void *stream);

/* -------------------------------------------------------------- utilities */

/* Synchronises `stream`, then copies the device status word of d_work into
 * *h_status (a vox_status value).  Returns VOX_ERR_DEVICE if a HIP call
 * fails. */
vox_status vox_read_status(const void *d_work, int32_t *h_status, void *stream);

/* Static description of a status code. */
const char *vox_status_string(vox_status status);

/* Message of the last host-side error on the calling thread ("" if none). */
const char *vox_last_error(void);

/* VOX_ABI_VERSION of the built library. */
int vox_abi_version(void);

/* ------------------------------------------------------- kernel timing */

/* Tracing of the library's own kernels.  While enabled, each kernel launch
 * of every entry point is bracketed by two HIP events recorded on the
 * launch's stream, and its duration is added to a per-kernel record.
 * Launches made while their stream is being captured into a graph are not
 * timed.  Process-wide and thread-safe. */
vox_status vox_profile_enable(int enable);

/* Drops all records (after waiting for pending events). */
void vox_profile_reset(void);

/* Number of per-kernel records. */
int vox_profile_count(void);

/* Record `index`: kernel name (copied into name[name_len]), summed
 * duration in milliseconds and number of launches.  Synchronises on every
 * pending event.  VOX_ERR_INVALID_ARGUMENT for a bad index. */
vox_status vox_profile_read(int index, char *name, size_t name_len, double *total_ms,
                            int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* VOX_H */
