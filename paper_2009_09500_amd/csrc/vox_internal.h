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
constexpr int32_t kStatusLaunch = 4;  // batch table does not fit the launch or workspace

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
constexpr int kListPerThread = 4;
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
constexpr int64_t kSegsPerRow = 4096;   // segments staged per histogram round

// One volume of a brick-path launch, as the kernels read it from the
// device scene table.
struct BrickScene {
    const int32_t* segs;   // [n][6], 8-byte aligned
    int32_t* counts;       // [n] or null
    uint32_t* grid;        // packed bit-volume
    int64_t n;
    uint64_t hist_off;     // this scene's histogram rows, in words
    BrickGeom bg;
    uint32_t brick_base;   // global id of the scene's first brick
    uint32_t row_base;     // global index of its first histogram row
    uint32_t rows;         // histogram rows (workgroups) of the scene
    uint32_t flags;        // kSceneClear
};
constexpr uint32_t kSceneClear = 1;

// Device scene table: this header, BrickScene[n_scenes] at kTableScenes,
// then (several scenes only) uint32 row_scene[rows] and uint32
// brick_scene[bricks], the scene of each histogram row and of each global
// brick.  Position independent: the host builds it, any copy works.
struct BrickTable {
    uint32_t magic;
    uint32_t n_scenes;
    uint32_t rows;
    uint32_t bricks;
    int32_t lg[3];
    uint32_t max_nb;       // largest per-scene brick count
    uint64_t hist_words;
    uint64_t pieces;       // piece-record capacity (worst case)
    uint64_t work_bytes;   // workspace the table needs
    uint64_t table_bytes;
};
constexpr uint32_t kTableMagic = 0x564F5842u;  // "BXOV"
constexpr size_t kTableScenes = 64;
static_assert(sizeof(BrickTable) <= kTableScenes, "table header fits its slot");

// Launch bounds of a brick-path launch sequence (host side).
struct BrickLaunch {
    uint32_t rows;
    uint32_t bricks;
    int32_t lg[3];
    uint32_t max_nb;
};

// Workspace: [status word, launch-ok flag, 8 brick queues] | the one-scene table of
// a plain call | histogram rows | brick totals | bin offsets | piece records.
constexpr size_t kWorkTable = kAlign;
constexpr size_t kWorkData = kAlign + 512;
static_assert(kTableScenes + 160 <= 512, "one-scene table fits its slot");

void default_brick_lg(int32_t dx, int32_t dy, int32_t dz, int lg[3]);
bool brick_shape_supported(const int lg[3]);
// brick_geometry (vox_exact.h) for host files that do not compile device code.
bool brick_geometry_for(int32_t dx, int32_t dy, int32_t dz, const int lg[3], BrickGeom& bg);
// Process-wide brick shape chosen with vox_set_tuning (all zero = default).
void tuned_brick_lg(int lg[3]);
uint64_t max_pieces(int64_t n, const BrickGeom& bg);
int hist_rows(int64_t n);
size_t brick_work_bytes(uint64_t hist_words, uint32_t bricks, uint64_t pieces);

// Fills the table header fields derived from the scenes (rows, bricks,
// hist_words, pieces, max_nb, work_bytes) and each scene's bases; false if
// a total overflows the 32-bit brick, row or piece indices.
bool brick_table_layout(BrickTable& t, BrickScene* scenes, uint32_t n_scenes);

// Launches the brick pipeline over the device table d_table.  For a plain
// call pass one_table/one_scene (the init kernel writes them into the
// workspace, d_table is ignored).
hipError_t launch_bricks(const void* d_table, const BrickLaunch& L, const BrickTable* one_table,
                         const BrickScene* one_scene, void* d_work, size_t work_bytes,
                         hipStream_t stream);
hipError_t launch_brick_grid(const int32_t* segs, int64_t n, const BrickGeom& bg,
                             uint32_t* grid, int32_t* counts, uint32_t flags, void* d_work,
                             size_t work_bytes, hipStream_t stream);
size_t brick_workspace_bytes(int64_t n, const BrickGeom& bg);

size_t grid_workspace_bytes(int64_t n, int32_t dx, int32_t dy, int32_t dz);
GridWork grid_workspace(void* d_work, size_t work_bytes, int64_t n, int32_t dx, int32_t dy, int32_t dz);

hipError_t launch_grid(const int32_t* segs, int64_t n, bool aligned8, int32_t dx, int32_t dy,
                       int32_t dz, uint32_t* grid, int32_t* counts, uint32_t flags,
                       const GridWork& w, hipStream_t stream);

}  // namespace vox
