// Internal layouts shared by the host side of the C ABI (sgn_api.cpp) and
// the HIP kernels (sgn_kernels.hip).  Not part of the public interface.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sgn {

constexpr int kMaxNbr = 16;
constexpr int kWaveSize = 64;
constexpr int kBlockThreads = 256;      // 4 wavefronts per workgroup
constexpr int kNumCounters = 16;        // work-queue heads (one per XCD + spares)
constexpr int kXcds = 8;

// Per-keyframe descriptor in device memory (one per batch item).
struct KfDev {
    const void* kf_img;
    float* inv_depth;
    float* nx;
    float* ny;
    float* nz;
    uint32_t* flags;
    float* cost;
    uint32_t* nvalid;
    uint32_t* last_update;
    const uint8_t* is_new;        // may be null
    float* inv_depth_out;         // may be null
    int32_t* index_out;           // may be null
    int32_t width, height, kf_pitch, n_nbr;
    int32_t gw, gh, frame_base, item_base;      // frames: [frame_base, frame_base + n_nbr)
    int32_t groups_x, n_items, surfel_base, queue;  // anchor blocks per row; work items
    int64_t pixel_base;                          // prefix over render segments (row x tile column)
    int32_t patch, nbr_pitch_b;                   // neighbour-image row pitch in bytes
    double fx_d, fy_d, cx_d, cy_d;               // intrinsics as given (double)
    float fx, fy, cx, cy;                        // the same, rounded to float
    float kf_scale, img_scale, pad0, pad1;
    // disc surfels (Eq. 4): centres of the surfels, radius in pixels; null
    // and 0 for tiles
    const float* disc_ux;
    const float* disc_uy;
    float disc_r;
    int32_t disc_count;           // surfels of the keyframe (an item is a run of them)
};

// Per-neighbour-frame descriptor.  R and t are the caller's pose in double;
// hm/kt are written on the device by the setup kernel.
struct FrameDev {
    float zrow[4];  // hm[6], hm[7], kt[2] rounded to float (the q_z row), pad
    const void* img;  // next to zrow: one scalar load per frame fetches both
    int32_t pitch, pad0;
    double R[9];
    double t[3];
    double hm[9];   // K R K^-1
    double kt[3];   // K t
};

// Work queue q covers the global item range [begin, end).
struct QueueDev {
    int32_t begin, end;
};

// Header of one batch, in device memory, read by every kernel.  All per-call
// values live here (not in kernel arguments) so that a captured graph can be
// replayed for any batch.
struct BatchHeader {
    KfDev* kfs;
    FrameDev* frames;
    int32_t n_kf, n_frames, total_items, total_surfels;
    int64_t total_pixels;           // render segments of the batch
    int32_t iters;
    float huber_k;
    float kappa_fp64;
    int32_t depth_only;
    float beta_r;
    uint32_t stamp;
    int32_t do_init, do_gn, do_render, n_queues;
    float lm_lambda;
    int32_t pad_lm;
    QueueDev queues[kNumCounters];
};

enum : uint32_t {
    F_DEGENERATE = 1u << 0,
    F_FEW_SAMPLES = 1u << 1,
    F_SOLVE_FAIL = 1u << 2,
    F_REJECTED = 1u << 3,
    F_FP64_SOLVE = 1u << 4,
    F_UNINIT = 1u << 5,
    F_GN_BITS = F_DEGENERATE | F_FEW_SAMPLES | F_SOLVE_FAIL | F_REJECTED | F_FP64_SOLVE,
};

// Kernel variants.
struct GnVariant {
    int dtype;      // 0 f32, 1 f16, 2 u8
    int patch;      // 4, 8 or 16
    int tiles_x, tiles_y;
    int lds;        // stage footprints in LDS
    int groups;     // surfel groups per work item (1, 2 or 4)
    int by_row;     // neighbour rows read by index (every row pitch below kMaxRowStride)
};
// Row pitch (bytes) up to which neighbour images are read through a
// structured buffer, the row as the index: the descriptor's stride field holds
// 14 bits.  Wider rows are read with raw byte offsets.
constexpr unsigned kMaxRowStride = 16384;

// Work-item geometry of the Gauss-Newton kernel.  Surfels are taken in
// aligned anchor blocks of 16 x 16 pixels (ab x ab tiles).  A work item is an
// ix x iy tile sub-block of one anchor block holding K groups of tx x ty
// tiles (one group fills a wavefront: four or eight 4 x 4 surfels, one 8 x 8
// or one 16 x 16 surfel), arranged gx x gy, as wide as the anchor block
// allows; ipb items tile an anchor block.
struct ItemGeo {
    int ab, gx, gy, ix, iy, ipb;
};
constexpr ItemGeo item_geo(int S, int TX, int TY, int K) {
    const int ab = 16 / S;
    const int gx = (S == 4) ? (K < 4 / TX ? K : 4 / TX) : (K >= 2 ? 2 : 1);
    const int gy = K / gx;
    const int ix = gx * TX, iy = gy * TY;
    return ItemGeo{ab, gx, gy, ix, iy, (ab / ix) * (ab / iy)};
}

// Arguments of the re-gridding kernels (Eq. 10).  Surfel arrays are device
// memory; best/win are scratch of one entry per destination tile.
struct RegridSurfels {
    float* inv_depth;
    float* nx;
    float* ny;
    float* nz;
    uint32_t* flags;
    float* cost;
    uint32_t* nvalid;
    uint32_t* last_update;
};
struct RegridArgs {
    RegridSurfels src, dst;
    double src_K[4], dst_K[4];   // fx, fy, cx, cy
    double R[9], t[3];           // X_dst = R X_src + t
    int32_t src_w, src_h, src_patch, dst_w, dst_h, dst_patch;
    unsigned long long* best;    // closest landing per destination tile (bits of 1/p'_z)
    int32_t* win;                // winning source index per destination tile
    uint8_t* is_new;
    int32_t* src_index;          // may be null
    int32_t dst_base;              // destination tiles of the table's earlier pairs (best, win offsets)
    int32_t src_count, dst_count;  // this pair's source surfels / destination tiles
    int32_t src_wave, dst_wave;    // this pair's first 64-lane wavefront over sources / tiles
};

// Launchers implemented in sgn_kernels.hip.  All return hipError_t of the
// launch.
hipError_t launch_setup(const BatchHeader* hdr, uint32_t* counters, int n_frames_cap,
                        hipStream_t s);
hipError_t launch_init(const BatchHeader* hdr, int grid, hipStream_t s);
hipError_t launch_render(const BatchHeader* hdr, int grid, hipStream_t s);
hipError_t launch_gn(const GnVariant& v, const BatchHeader* hdr, uint32_t* counters,
                     int persistent, int grid_blocks, hipStream_t s);
// Device address of the static scratch array on `device` (which must be the
// current device), looked up on the first call for that device and kept.
hipError_t static_scratch_on(int device, void** out);
// Re-gridding of a device table of n_pairs keyframe pairs.  A wavefront
// never spans two pairs: pair k's sources run over the
// wavefronts from src_wave on (surfel i at lane i % 64 of wavefront
// src_wave + i / 64), likewise its tiles from dst_wave; src_waves and
// dst_waves are the totals.
hipError_t launch_regrid(const RegridArgs* table, int n_pairs, int src_waves, int dst_waves,
                         hipStream_t s);

// Disc surfels (Eq. 4).
constexpr float kDiscMaxRadius = 12.f;
// Disc surfels per wavefront of the Gauss-Newton kernel, by image type
// (0 f32, 1 f16, 2 u8): two (32 lanes each) where a pixel's LDS slot packs
// into one word, one for f32 images.
constexpr int disc_surfels_per_wave(int dtype) { return dtype == 0 ? 1 : 2; }
// Gauss-Newton over the disc surfels of a batch: one wavefront per work item
// of disc_surfels_per_wave(dtype) surfels of one keyframe (KfDev::n_items =
// ceil(disc_count / that), item_base their prefix).
// grid_blocks workgroups of four wavefronts, one work item each (with one
// share per XCD in the header, workgroup b serves share b % kXcds)
hipError_t launch_disc_gn(int dtype, const BatchHeader* hdr, int total_items, int grid_blocks, bool by_row,
                          hipStream_t s);
// Depth-buffered render of the discs of several keyframes: one table entry
// per keyframe (device memory); the scratch holds one 64-bit depth key and
// one index per pixel of every keyframe, keyframe after keyframe.
struct DiscRenderItem {
    const float* inv_depth;
    const float* nx;
    const float* ny;
    const float* nz;
    const uint32_t* flags;
    const float* ux;
    const float* uy;
    float* inv_depth_out;         // [width * height]
    int32_t* index_out;           // [width * height] or null
    int32_t count, width, height, surfel_base;
    int64_t pixel_base;
    float radius;
    int32_t tiles_x;              // render tiles per row (kRenderTile pixels square)
    double fx, fy, cx, cy;
    int32_t tile_base;            // render tiles of the table's earlier keyframes
    int32_t pad;
};
constexpr int kRenderTile = 16;
// Per usable surfel: centre, normal and the denominator of Eq. 3, in double.
struct DiscRaster {
    double cx, cy, n0, n1, n2, den;
};
// The render's scratch: raster records [surfels], tile counts [tiles], list
// starts [tiles + 1], scan block sums [ceil(tiles / 1024)], tile lists
// [kDiscMaxTilesPerSurfel * surfels].
constexpr int kDiscMaxTilesPerSurfel = 9;     // a box of <= 2 r + 1 <= 25 pixels meets <= 3 x 3 tiles
struct DiscRenderScratch {
    DiscRaster* rec;
    int32_t* count;
    int32_t* start;
    int32_t* block_sum;
    int32_t* list;
};
hipError_t launch_disc_render(const DiscRenderItem* table, int n_items, int total_surfels, int total_tiles,
                              const DiscRenderScratch& w, hipStream_t s);
// The search for empty areas on the lattice (spacing/2 + i spacing, ...),
// placement of the qualifying candidates as surfels first .. and their
// neighbour initialisation from the index map.
struct DiscPlaceArgs {
    float* inv_depth;
    float* nx;
    float* ny;
    float* nz;
    uint32_t* flags;
    float* cost;
    uint32_t* nvalid;
    uint32_t* last_update;
    float* ux;
    float* uy;
    const int32_t* index_map;     // [width * height]
    int32_t first, room;          // existing surfels; free entries after them
    int32_t width, height, spacing, cand_x, cand_y;   // lattice of cand_x x cand_y candidates
    float radius, alpha, beta;
    float fx, fy, cx, cy;
    uint8_t* cand_flag;           // scratch [cand_x * cand_y]
    int32_t* counts;              // device [2]: placed, qualifying
    int32_t cand_base;            // candidates of the table's earlier keyframes
    int32_t init_base;            // new-surfel slots (min(room, candidates)) of earlier keyframes
};
// Placement for a device table of n_items keyframes: search (one wavefront
// per candidate), compaction (one workgroup per keyframe), initialisation
// (one wavefront per new-surfel slot).
hipError_t launch_disc_place(const DiscPlaceArgs* table, int n_items, int total_cands, int total_init,
                             hipStream_t s);
// Eq. 10 for disc surfels: each usable source surfel moves to p' = R p + t,
// n' = R n, and is re-centred at K_dst pi(p'); those landing in the
// destination image are written in source order.
struct DiscTransferArgs {
    const float* inv_depth;
    const float* nx;
    const float* ny;
    const float* nz;
    const uint32_t* flags;
    const uint32_t* last_update;
    const float* ux;
    const float* uy;
    int32_t count, dst_w, dst_h, capacity;
    double sK[4], dK[4];          // fx, fy, cx, cy of source and destination
    double R[9], t[3];            // X_dst = R X_src + t
    RegridSurfels dst;
    float* dux;
    float* duy;
    int32_t* src_index;           // may be null
    int32_t* counts;              // device [2]: written, landed
};
// One workgroup per entry of a device table of n_pairs keyframe pairs.
hipError_t launch_disc_transfer(const DiscTransferArgs* table, int n_pairs, hipStream_t s);
hipError_t launch_quantize(const float* src, int src_pitch, void* dst, int dst_pitch,
                           int width, int height, int dtype, float scale, hipStream_t s);
// Workgroups of 256 threads of the chosen GN variant that fit on one CU.
int gn_blocks_per_cu(const GnVariant& v);
bool gn_variant_supported(const GnVariant& v);

}  // namespace sgn
