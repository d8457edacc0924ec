// Host-side launch interface between the C ABI layer (vox_api.cpp) and the
// kernel files.  Internal; not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vox {

// Device status word bits (first int32 of every workspace).  The host maps
// the set bits onto a vox_status code.
constexpr int32_t kStatusOutOfRange = 1;
constexpr int32_t kStatusCapacity = 2;
constexpr int32_t kStatusLaunch = 4;  // batch scenes exceed the launch bounds (n_scenes / total_segments)
constexpr int32_t kStatusInvalid = 8; // a batch scene breaks an argument rule

// Scoped kernel timer: records HIP events on `stream` around the launch
// made inside its scope when kernel timing is enabled (vox_profile_enable);
// otherwise does nothing.  Names must be string literals.
class KernelTimer {
  public:
    KernelTimer(const char* name, hipStream_t stream);
    ~KernelTimer();
    KernelTimer(const KernelTimer&) = delete;
    KernelTimer& operator=(const KernelTimer&) = delete;

  private:
    const char* name_;
    hipStream_t stream_;
    hipEvent_t start_ = nullptr;
};

// Sets the calling thread's last-error message (vox_last_error) and returns
// `status` (a vox_status value).
int report_error(int status, const char* fmt, ...);

// Workspace sections are 256-byte aligned.
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------- list path
// Segment blocks of the count/offset kernels and voxel tiles of the list
// kernel.
constexpr int kCountBlock = 256;
constexpr int kCountPerThread = 4;
constexpr int64_t kSegsPerCountBlock = (int64_t)kCountBlock * kCountPerThread;
constexpr int kListBlock = 256;
constexpr int kListPerThread = 8;
constexpr int64_t kListTile = (int64_t)kListBlock * kListPerThread;

struct ListWork {
    int32_t* status;       // [1]
    int64_t* total;        // [1]
    int64_t* block_sums;   // [nb]  block totals, then block prefixes
    int32_t* block_flags;  // [nb]
    uint32_t* counts;      // [n]
    int32_t* tile_seg;     // [ntiles + 1]
    int64_t nb;
    int64_t ntiles;
};

size_t list_workspace_bytes(int64_t n, int64_t capacity);
ListWork list_workspace(void* d_work, int64_t n, int64_t capacity);

// The list forms: int16 coordinates with the Chebyshev N; int16 with the
// Euclidean N of eq. (1); int32 coordinates with the Chebyshev N.
enum ListKind { kListI16 = 0, kListEuclid = 1, kListI32 = 2 };

hipError_t launch_list_count(const int32_t* segs, int64_t n, bool aligned8, const ListWork& w,
                             hipStream_t stream, ListKind kind);
// Count, scan and offsets in one block, for 1 <= n <= kSegsPerCountBlock.
hipError_t launch_list_one_block(const int32_t* segs, int64_t n, bool aligned8, const ListWork& w,
                                 int64_t* offsets, int64_t capacity, bool want_voxels, hipStream_t stream,
                                 ListKind kind);
hipError_t launch_list_scan(const ListWork& w, int64_t n, int64_t* offsets, int64_t capacity,
                            bool want_voxels, hipStream_t stream);
hipError_t launch_list_offsets(int64_t n, int64_t* offsets, const ListWork& w, int64_t capacity,
                               bool want_voxels, hipStream_t stream);
hipError_t launch_list_voxels(const int32_t* segs, int64_t n, bool aligned8, const int64_t* offsets,
                              const ListWork& w, int16_t* voxels, int64_t capacity,
                              int64_t tiles_to_launch, hipStream_t stream);
hipError_t launch_list_voxels32(const int32_t* segs, int64_t n, bool aligned8, const int64_t* offsets,
                                const ListWork& w, int32_t* voxels, int64_t tiles_to_launch, hipStream_t stream);
hipError_t launch_list_voxels_euclid(const int32_t* segs, int64_t n, bool aligned8, const int64_t* offsets,
                                     const ListWork& w, int16_t* voxels, hipStream_t stream);

// ------------------------------------------------------------- grid path
struct GridWork {
    int32_t* status;  // first word of the workspace
    size_t bytes;     // workspace size
};

// Brick decomposition of a volume: bricks of 2^lg[a] voxels per axis,
// nb[a] bricks per axis (edge bricks may be partial), brick id
// (bz * nb[1] + by) * nb[0] + bx.
struct BrickGeom {
    int32_t dim[3];
    int32_t lg[3];
    int32_t nb[3];
    uint32_t nbricks;
};

constexpr uint32_t kMaxBricks = 16384;  // LDS histogram of 64 KiB
constexpr int kHistBlock = 1024;
constexpr int kHistRows = 256;
// Segments per histogram row (one workgroup of the histogram and scatter
// kernels): a batch has the parallelism of its many scenes and keeps its
// workspace bound small with 4096; a plain call of one volume takes rows of
// 512, so that a call of a few hundred thousand segments still spreads over
// the CUs (both reach the 256 rows a scene may have at large n).
constexpr int64_t kSegsPerRow = 4096;
constexpr int64_t kSegsPerRowPlain = 512;

// One volume of a launch as the kernels read it from the device scene table
// (written by the plan kernel from the caller's vox_scene entries).
struct BrickScene {
    const int32_t* segs;   // [n][6]
    int32_t* counts;       // [n] or null
    uint32_t* grid;        // packed bit-volume
    int64_t n;
    uint64_t hist_off;     // brick scenes: histogram rows, in words; direct scenes: first segment
                           // among the direct scenes' segments
    BrickGeom bg;          // brick scenes only (dim[] always)
    uint32_t brick_base;   // global id of the scene's first brick
    uint32_t row_base;     // global index of its first histogram row
    uint32_t rows;         // histogram rows (workgroups) of the scene; 0 for a direct scene
    uint32_t flags;        // kScene*
};
constexpr uint32_t kSceneClear = 1;    // zero the volume first
constexpr uint32_t kSceneDirect = 2;   // the direct kernels serve this scene (no bricks)
constexpr uint32_t kSceneEuclid = 4;   // Euclidean N of eq. (1)
constexpr uint32_t kSceneA8 = 8;       // segment array 8-byte aligned

// Device scene table, written into the workspace by the plan kernel: this
// header, BrickScene[n_scenes] at kTableScenes, then uint32 direct[n_scenes]
// (the direct scenes in order), and with several scenes uint32
// row_scene[rows bound] and uint32 brick_scene[bricks bound]: the scene of
// each histogram row and of each global brick.
struct BrickTable {
    uint32_t magic;
    uint32_t n_scenes;
    uint32_t rows;         // histogram rows of all brick scenes
    uint32_t bricks;       // bricks of all brick scenes
    int32_t lg[3];
    uint32_t max_nb;       // largest per-scene brick count
    uint64_t hist_words;
    uint64_t data_off;     // workspace offset of the histograms (then totals, offsets, records)
    uint32_t n_direct;     // scenes served by the direct kernels
    uint32_t row_cap;      // entries of row_scene
    uint64_t direct_segs;  // segments of the direct scenes
};
constexpr uint32_t kTableMagic = 0x564F5842u;  // "BXOV"
constexpr size_t kTableScenes = 64;
static_assert(sizeof(BrickTable) <= kTableScenes, "table header fits its slot");

// Workspace header words (int32 / uint32 index into the first 256 bytes).
constexpr int kWStatus = 0;    // status bits (kStatus*)
constexpr int kWOk = 2;        // 1 when the brick kernels may run
constexpr int kWDirectAll = 3; // 1: the direct kernels serve every scene (records do not fit)
constexpr int kWQueues = 4;    // 8 work queues of the fill
constexpr int kWItems = 12;    // the fill's work items (k_brick_base)
constexpr int kWSplit = 13;    // bricks cut into several work items (k_brick_base)
constexpr int kWPieces = 16;   // uint64: piece records the call needed (information)
constexpr size_t kWorkTable = kAlign;

// Launch bounds of a brick-path launch sequence (host side): the kernels
// are sized by these, and the plan kernel checks that the scenes stay
// within them.
struct BrickLaunch {
    uint32_t n_scenes;
    uint64_t total_segments;  // bound on the scenes' segments
    uint32_t rows;            // histogram rows bound
    uint32_t bricks;          // bricks bound
    int32_t lg[3];
    uint64_t table_bytes;     // table region (bound)
    bool direct_kernels;      // launch the direct kernels (some scene may need them)
    uint32_t segs_per_row;    // kSegsPerRow or kSegsPerRowPlain
};

// Histogram rows of a brick scene of n segments, per_row segments a row.
__host__ __device__ inline uint32_t hist_rows(int64_t n, int64_t per_row) {
    int64_t g = (n + per_row - 1) / per_row;
    if (g > kHistRows) g = kHistRows;
    if (g < 1) g = 1;
    return (uint32_t)g;
}

void default_brick_lg(int32_t dx, int32_t dy, int32_t dz, int lg[3]);
bool brick_shape_supported(const int lg[3]);
// brick_geometry (vox_exact.h) for host files that do not compile device code.
bool brick_geometry_for(int32_t dx, int32_t dy, int32_t dz, const int lg[3], BrickGeom& bg);
// Worst case of piece records of n segments in a volume.
uint64_t max_pieces(int64_t n, const BrickGeom& bg);

// Launch bounds of a batch of n_scenes scenes holding at most
// total_segments segments, for bricks of 2^lg, and the workspace bytes
// before the piece records (table, histograms, brick totals and offsets).
BrickLaunch batch_launch(uint32_t n_scenes, uint64_t total_segments, const int lg[3]);
size_t batch_fixed_bytes(const BrickLaunch& L);
constexpr uint64_t kRecordBytes = 16;
constexpr uint64_t kDefaultPiecesPerSegment = 16;

// Launches the brick pipeline over the scenes d_scenes[n_scenes] (device
// vox_scene array, planned by the plan kernel), or over the single scene
// *one (a host vox_scene, planned inside the histogram launch) when
// d_scenes is null.
hipError_t launch_bricks(const void* d_scenes, const void* one, const BrickLaunch& L, int fill_wgs_per_cu,
                         void* d_work, size_t work_bytes, hipStream_t stream);
// Launch bounds of a plain call that takes the brick path, and its
// workspace: the fixed part plus room for the worst case of records.
BrickLaunch plain_launch(int64_t n, const BrickGeom& bg);
size_t brick_workspace_bytes(int64_t n, const BrickGeom& bg);

size_t grid_workspace_bytes(int64_t n, int32_t dx, int32_t dy, int32_t dz);
// The part of a compact workspace a plain call needs before its records (the
// brick path runs as a one-scene batch in a smaller workspace).
size_t grid_compact_fixed_bytes(int64_t n, int32_t dx, int32_t dy, int32_t dz);
GridWork grid_workspace(void* d_work, size_t work_bytes, int64_t n, int32_t dx, int32_t dy, int32_t dz);

hipError_t launch_grid(const int32_t* segs, int64_t n, bool aligned8, int32_t dx, int32_t dy,
                       int32_t dz, uint32_t* grid, int32_t* counts, uint32_t flags,
                       const GridWork& w, hipStream_t stream);

// Tuning: the per-call choice, else the library's autotune cache for the
// key (volume, segment count), else the default.  `valid` rejects shapes
// without a compiled kernel and non-zero reserved fields.
struct Tuning {
    int lg[3];
    int fill_wgs_per_cu;  // 0 = the shape's default
};
bool tuning_from_abi(const void* vox_tuning_ptr, Tuning& t, char* why, size_t why_len);
bool tuning_cache_lookup(int32_t dx, int32_t dy, int32_t dz, int64_t n, Tuning& t);

}  // namespace vox
