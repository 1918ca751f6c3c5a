// Internal layout shared by the host part and the kernels of liblidarseg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lidarseg.h"

namespace lidarseg {

constexpr uint64_t KEY_EMPTY = ~0ull;
constexpr int MAX_RINGS = 128;
constexpr int POINT_BLOCK = 1024;            // points per binning work item
constexpr int VITEM = 1024;                  // vertex slots per labelling work item
constexpr int VITEM_WORDS = VITEM / 64;      // 64-bit root-flag words per labelling item
constexpr int64_t MAX_CELLS = 1ll << 29;     // per frame; keeps every count below 2^30
constexpr int64_t MAX_BATCH_CELLS = (1ll << 31) - VITEM;  // forest positions are int32
constexpr int MAX_TILE_CELLS = 2048;
constexpr int OCC_WORDS = MAX_TILE_CELLS / 64;        // occupancy words per tile
constexpr int MAX_SCORE_RADIUS = 8;          // dilation radius of the edge scores

// One frame of a batch, as the kernels see it.  Lives in device memory right
// after a BatchHeader; all offsets index the context's workspace arrays.
struct FrameDesc {
    const float* xyz;         // [n_points][3]
    const float* normals_in;  // optional per-vertex normals to label instead
    float* vertices;
    float* normals;
    int32_t* labels;
    int32_t* tris;
    int32_t* vpoint;          // may be null
    int64_t* counts;
    int32_t* point_labels;    // may be null: every input point's label
    const int32_t* truth;     // may be null: ground-truth surface id per input point
    const uint8_t* rings;     // may be null: the reported ring of each input point
    int64_t* scores;          // may be null: the frame's edge counts (needs truth)
    int64_t n_points;
    int64_t cell_off;         // first cell of this frame in the key grid and the forest
    int64_t border_off;       // first border slot (int2) of this frame: 2H slots per tile
    int64_t pt_off;           // first per-point record of this frame (when point_labels)
    int32_t H, W, s, Wp, wrap, TW;
    int32_t n_tiles, tile_off;
    int32_t n_pblk, pblk_off;
    int32_t n_vitem, vitem_off;  // labelling items (VITEM vertex slots each); words at vitem_off * VITEM_WORDS
    int32_t elev_off;
    int32_t pred;             // similarity test: 0 components (Algorithm 1), 1 cosine
    int32_t min_seg;          // >= 2: segments with fewer vertices get label 0
    int32_t score_r;          // dilation radius of the edge scores
    double az0, dphi, rmin2, rmax2;
    double thr[3];
    double cos_min;
};

struct BatchHeader {
    int32_t n_frames;
    int32_t total_tiles;
    int32_t total_pblk;
    int32_t total_vitems;
    int32_t total_border;     // border slots of the batch
    int32_t post;             // 1: some frame asks for segment removal or point labels
    FrameDesc* frames() { return reinterpret_cast<FrameDesc*>(this + 1); }
};
static_assert(sizeof(BatchHeader) == 24, "header size");
static_assert(sizeof(FrameDesc) % 8 == 0, "desc alignment");

// Device workspace of a context.  Per-tile arrays are indexed by the batch-wide
// tile index; keys and forest by cell_off + cell (firing order within a frame),
// the forest's entries being batch-wide positions cell_off + vertex.
struct Workspace {
    uint64_t* keys;       // (float(r^2) bits << 32) | point index; KEY_EMPTY = no point
    int32_t* forest;      // union-find parent of each vertex, as a batch-wide position
    int32_t* tile_v;      // vertices owned by each tile
    int32_t* tile_t;      // triangles anchored in each tile
    int32_t* tile_vbase;  // vertices of the frame's tiles before each tile (written by k_geom)
    uint64_t* occ;        // per tile, OCC_WORDS words: occupancy of its own cells (bit l of
                          // the tile's cell sequence, firing order from its first column)
    uint64_t* rootbits;   // per 64 vertex slots: which vertices are segment roots
    uint32_t* wprefix;    // per 64 vertex slots: roots of its labelling item before the word
    int32_t* vitem_roots; // per labelling item: its roots, then (after k_scan) the roots
                          // of the frame before it
    int2* border;         // per tile and ring: the similar C and B joins that leave the
                          // tile through its right edge (forest positions), or (-1, -1)
    int32_t* pcell;       // per input point (pt_off + p): j * H + i of its full-resolution
                          // ring i and firing j, -1 if not used (point labels only)
    int32_t* cvid;        // per cell (cell_off + cell): its vertex id, -1 if empty (point labels only)
    int32_t* segsize;     // per label (cell_off + label - 1): vertices carrying it (segment removal)
    int32_t* vtruth;      // per vertex (cell_off + vertex): truth id of its point (edge scores)
    const double* elev;   // ring elevations, per frame at elev_off
};

// Tile geometry: a tile is TW consecutive sampled columns, all H rings.
inline int tile_width(int H, int tile_cells) {
    int tw = tile_cells / H;
    return tw < 1 ? 1 : tw;
}

constexpr int N_STAGES = 11;  // bin, count, geom, cc, merge, compress, flatten, scan, label, post, score

struct LaunchCfg {
    int grid;        // workgroups for grid-stride stages
    int tile_cells;  // 512, 1024 or 2048
    int tile_threads;  // 256 or 512 threads per tile workgroup
    int max_tiles;   // tiles in the largest batch this chain may see (for exact grids)
    int max_pblk;
    int max_vitems;
    int max_border;  // border slots
    int max_frames;
    bool post = false;   // launch the segment-removal / point-label stage
    bool score = false;  // launch the edge-score stage
    bool mesh_only = false;  // binning, mesh and normals only (no labelling stages)
    int stage_grid[N_STAGES] = {};  // per stage: workgroups, 0 = from grid
};


// Tile shapes (cells per tile, threads per tile workgroup) the kernels are built for.
bool tile_shape_supported(int tile_cells, int tile_threads);

// Sets n keys to KEY_EMPTY with a fill kernel (not a memset node, so the fill
// also behaves when a caller captures it into a graph).
hipError_t fill_keys_empty(uint64_t* keys, int64_t n, hipStream_t stream);

// Enqueues the chain; when stage_events is non-null (N_STAGES + 1 events) an
// event is recorded before the first kernel and after each kernel.
hipError_t launch_chain(const BatchHeader* d_hdr, const Workspace& ws, const LaunchCfg& cfg,
                        hipStream_t stream, hipEvent_t* stage_events = nullptr);

// Grows ctx's workspace up front so that no call of at most max_frames
// sweeps of these sensors whose device bytes (bytes_per_sensor[s] each) sum to
// at most budget (0 = no budget) has to grow it later, in the batched and graph
// forms or (plain) in the plain form.  Growth waits for the device, which a
// server must not do while it serves.
int ctx_reserve(lidar_ctx* ctx, const lidar_sensor_t* sensors, int32_t n_sensors, int32_t max_frames,
                uint64_t budget, const uint64_t* bytes_per_sensor, bool plain, hipStream_t stream);

}  // namespace lidarseg
