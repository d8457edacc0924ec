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
 *     first int32 of d_work, as VOX_DEVICE_STATUS_* bits; vox_read_status()
 *     fetches it as a vox_status code, vox_device_status() gives its device
 *     address.  Such errors never cause an out-of-bounds write: the affected
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

#define VOX_ABI_VERSION 6

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
    VOX_ERR_BATCH_MISMATCH = 6    /* batch scenes exceed the call's bounds */
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

/* The lists of vox_segments_to_list with no workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  The workspace is
 * a 32 MiB device array the library holds on each GPU it runs on (from
 * module load to the end of the process); the call allocates nothing.
 * Every call on one GPU shares that GPU's array, so calls that overlap on
 * one GPU (different streams, or threads without ordering) race: order
 * them.  Arguments, output, errors and the h_total synchronisation are those
 * of vox_segments_to_list; device-found errors are reported only through
 * h_total (the status word lives in the library's array).  Calls whose
 * workspace, vox_list_workspace_bytes(n, capacity), exceeds 32 MiB (about
 * 7 million segments, fewer with a large capacity) return VOX_ERR_WORKSPACE
 * and launch nothing. */
vox_status vox_segments_to_list_noalloc(const vox_segment *d_segs, int64_t n,
                                        int64_t *d_offsets, int16_t *d_voxels,
                                        int64_t capacity, int64_t *h_total, void *stream);

/* ----------------------------------------------------------------- grids */

/* Workspace bytes for vox_segments_to_grid with n segments and the given
 * volume (the bound covers the worst case of every segment crossing the
 * whole volume).  A call also accepts the smaller compact workspace of
 * vox_workspace_bytes(VOX_OP_GRID, n, 1); see vox_segments_to_grid. */
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
 *   d_work     workspace, 256-byte aligned: vox_grid_workspace_bytes(...)
 *              bytes, or at least vox_workspace_bytes(VOX_OP_GRID, n, 1)
 *              (compact: room for 16 piece records a segment; a call whose
 *              records need more is served by the direct kernels instead,
 *              with the same output, and reports no error).
 *
 * Device-checked: both end points of a segment must lie inside the volume
 * (then every voxel does, as each coordinate is rounded from a value between
 * two in-range integers).  A segment that fails sets VOX_ERR_OUT_OF_RANGE
 * and contributes no voxel; the others are still written.
 *
 * Calls with more than 16384 segments, 8-byte-aligned d_segs, dim_x a
 * multiple of 32 and every side at most 16384 (and a brick count within the
 * library's limit; with VOX_GRID_EUCLID also a volume diagonal
 * sqrt((dim_x-1)^2 + (dim_y-1)^2 + (dim_z-1)^2) below 16385) fill LDS
 * bricks; the others take the direct path (one device atomic per voxel).
 * The output is the same. */
vox_status vox_segments_to_grid(const vox_segment *d_segs, int64_t n,
                                int32_t dim_x, int32_t dim_y, int32_t dim_z,
                                uint32_t *d_grid, int32_t *d_counts, uint32_t flags,
                                void *d_work, size_t work_bytes, void *stream);

/* ----------------------------------------------------------------- tuning */

/* Launch-shape choice for bit-volume calls (the build's counterpart of the
 * launch-shape options of Section 5: how the many segments of one call are
 * spread over the GPU).  brick_lg[a] is log2 of the LDS brick size along
 * axis a; all zero selects the library default.  The choice changes only
 * speed and workspace size, never the output.  Supported shapes:
 * 2^8 x 2^6 x 2^5, 2^8 x 2^6 x 2^6, 2^7 x 2^6 x 2^6, 2^7 x 2^7 x 2^6.
 * fill_wgs_per_cu: fill workgroups per compute unit: 1 (one of 1024
 * threads) or 2 (two of 512) for 64 KiB bricks, 1 for 128 KiB bricks; 0 =
 * the default (64 KiB bricks: 2, or 1 when the launch has fewer bricks than
 * two per compute unit).  reserved: zero. */
typedef struct vox_tuning {
    int32_t brick_lg[3];
    int32_t fill_wgs_per_cu;
    int32_t reserved[4];
} vox_tuning;

/* The library's autotune cache (process-wide, guarded by a mutex): the
 * tuning that vox_segments_to_grid uses for a volume of dim_x x dim_y x
 * dim_z and a segment count with the same floor(log2(n)), and that
 * vox_batch_scenes uses when it is passed no tuning (key dims 0 x 0 x 0 and
 * n = total_segments).  tuning NULL removes the entry.  Workspace sizes of
 * plain calls depend on it: query them after setting it.
 * VOX_ERR_INVALID_ARGUMENT for an unsupported tuning. */
vox_status vox_tuning_cache_set(int32_t dim_x, int32_t dim_y, int32_t dim_z, int64_t n_segments,
                                const vox_tuning *tuning);

/* The cache entry for a key: *found = 1 and *tuning filled, or *found = 0. */
vox_status vox_tuning_cache_get(int32_t dim_x, int32_t dim_y, int32_t dim_z, int64_t n_segments,
                                vox_tuning *tuning, int32_t *found);

/* Empties the autotune cache. */
void vox_tuning_cache_clear(void);

/* ---------------------------------------------------------------- batches */

/* One scene of a batch: its own segments and its own bit-volume, with the
 * meaning and the rules of the vox_segments_to_grid arguments of the same
 * names (flags: VOX_GRID_CLEAR and/or VOX_GRID_EUCLID).  48 bytes; an array
 * of them lives in device memory. */
typedef struct vox_scene {
    const vox_segment *segs; /* device; may be NULL if n == 0 */
    int64_t n;
    int32_t dim_x, dim_y, dim_z;
    uint32_t flags;
    uint32_t *grid;          /* device, 16-byte aligned */
    int32_t *counts;         /* device, optional (NULL) */
} vox_scene;

/* Operation codes of vox_workspace_bytes. */
#define VOX_OP_GRID 2
#define VOX_OP_BATCH 3

/* Workspace bytes for an operation, from the sizes known before the call:
 *   VOX_OP_GRID   the compact workspace of vox_segments_to_grid with n
 *                 segments in any volume (n_scenes must be 1): the
 *                 one-scene case of VOX_OP_BATCH below.
 *   VOX_OP_BATCH  vox_batch_scenes with n_scenes scenes of at most
 *                 n_segments segments in all.  The bytes hold the scene
 *                 table, the brick histograms, brick totals and offsets for
 *                 any scenes, and piece records for an average of 16 per
 *                 segment (a piece is a segment's run of voxels inside one
 *                 LDS brick: about 1 + N/32 for a segment of N steps).
 * 0 for an unknown op or negative sizes.  (Single-call workspaces:
 * vox_list_workspace_bytes, vox_grid_workspace_bytes.) */
size_t vox_workspace_bytes(int op, int64_t n_segments, int32_t n_scenes);

/* All scenes of a batch in one launch sequence, every kernel a single
 * launch over all scenes (the paper's advice to cut the number of kernel
 * calls and load the GPU with many segments at once, Section 4: all
 * segments in one core function call; Section 5, conclusions), the bricks of
 * all scenes taken by persistent workgroups from work-stealing queues.  Every
 * scene's grid (and counts) ends up exactly as a separate
 * vox_segments_to_grid call would leave it; the device status word covers
 * all scenes.
 *
 *   d_scenes        [n_scenes] vox_scene, device memory (read by the GPU
 *                   only), n_scenes in [1, 65536].
 *   total_segments  an upper bound on the sum of the scenes' n (sizes the
 *                   launch), >= 0.
 *   tuning          host struct, or NULL: the autotune cache entry for
 *                   (0 x 0 x 0, total_segments), else the default.
 *   d_work          workspace, 256-byte aligned, at least
 *                   vox_workspace_bytes(VOX_OP_BATCH, total_segments, n_scenes)
 *                   for full speed; see below.
 *
 * A plan kernel reads the scenes on the GPU and checks them against the
 * vox_segments_to_grid rules: a scene that breaks one, or scenes whose
 * segments exceed total_segments, stop the call with nothing written and
 * the status VOX_ERR_INVALID_ARGUMENT / VOX_ERR_BATCH_MISMATCH.  Scenes whose
 * segment array is 8-byte aligned, dim_x a multiple of 32, every side at
 * most 16384 and at most 16384 bricks (with VOX_GRID_EUCLID, a volume
 * diagonal below 16385) take the LDS brick kernels; the others (and every
 * scene, when the piece records of the call do not fit the workspace) take
 * direct kernels with one device atomic per voxel.  The output never depends
 * on which.
 *
 * Reads no device memory on the host, synchronises nothing and allocates
 * nothing, so it can be captured into a HIP graph once and replayed after
 * the caller rewrites d_scenes (same address, same n_scenes, segments within
 * total_segments).  Host-checked errors (returned, nothing launched): NULL
 * or misaligned d_scenes / d_work, n_scenes or total_segments out of range,
 * an unsupported tuning, a workspace smaller than the table and histogram
 * part of vox_workspace_bytes (VOX_ERR_WORKSPACE). */
vox_status vox_batch_scenes(const vox_scene *d_scenes, int32_t n_scenes, int64_t total_segments,
                            const vox_tuning *tuning, void *d_work, size_t work_bytes, void *stream);

/* -------------------------------------------------------------- utilities */

/* Bits of the device status word (first int32 of every workspace). */
#define VOX_DEVICE_STATUS_OUT_OF_RANGE 1u   /* an end point outside the output range */
#define VOX_DEVICE_STATUS_CAPACITY 2u       /* voxel list larger than the capacity   */
#define VOX_DEVICE_STATUS_MISMATCH 4u       /* batch scenes exceed the call's bounds */
#define VOX_DEVICE_STATUS_INVALID 8u        /* a batch scene breaks an argument rule */

/* Device address of the status word of a workspace (its first int32), for
 * callers that read or copy it in stream order themselves (a graph, a
 * serving loop copying it per batch).  0 after a call without device-found
 * errors, else the VOX_DEVICE_STATUS_* bits; every call rewrites it.  No
 * device access is made; NULL for NULL. */
int32_t *vox_device_status(void *d_work);

/* Synchronises `stream`, then reads from the workspace of the last
 * vox_batch_scenes (or brick-path vox_segments_to_grid) call: *h_pieces, the
 * piece records it needed, and *h_direct_all, 1 when they did not fit the
 * workspace and the direct kernels served every scene (the output is the
 * same; a workspace of the table and histogram part plus 16 bytes a record
 * avoids it).  Either pointer may be NULL.  VOX_ERR_DEVICE if a HIP call
 * fails. */
vox_status vox_read_batch_info(const void *d_work, uint64_t *h_pieces, int32_t *h_direct_all, void *stream);

/* Synchronises `stream`, then copies the device status word of d_work into
 * *h_status as a vox_status value (MISMATCH before INVALID before
 * OUT_OF_RANGE before CAPACITY).  Returns VOX_ERR_DEVICE if a HIP call
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
