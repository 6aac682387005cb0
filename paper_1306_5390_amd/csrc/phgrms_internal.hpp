// phgrms_internal.hpp -- declarations shared by the host-side sources of the
// library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "phgrms.h"
#include "host_common.hpp"

namespace phg {

constexpr int kDefaultShape = 3;   // (1, 8, 4): one pass, 8 rows per wave, 4 waves
// Launches at the start of a change-tracking pass loop that run the dense
// kernel of kDefaultShape (no change maps).  At most 2: the list-building
// launch of a skipping shape is launch 2.
constexpr int kDenseFirstLaunches = 2;
// Workgroups of a launch over listed tiles, in multiples of the grid that
// fits on the device at once.
constexpr int kListedOversubscription = 4;
// Largest grid (in workgroups of `threads` lanes) of a launch: fewer than
// 2^31 work-items per dispatch (the dispatch size stays a positive 32-bit
// count), a multiple of 16.  Only images near 2^31 pixels reach it; the
// tile-walking kernels take the tiles beyond the grid in strides.
inline long long max_workgroups(int threads) { return (0x7fffffffll / threads) / 16 * 16; }

struct TileGeom {
  int T;             // passes per launch
  int TH, TW;        // owned tile rows and columns
  int tiles_x, tiles_y;
  long long ntiles;
};
TileGeom tile_geom(const phgrms_params& p, int shape);

struct WsLayout {
  size_t state_off;    // int32 iteration count
  size_t counts_off;   // uint64 count slots, kCountSlots per pass
  size_t diff_off;     // uint64 slots of the period-2 stop, right after the counts
  size_t changed_off;  // uint64 changed[max(k,1)] totals
  size_t img_off;      // rows*cols bytes, the second ping-pong image
  size_t map_off;      // two change maps of map_bytes / 2 each
  size_t map_bytes;
  size_t total;
};
// Change maps of one-pass launches: one byte per (row, 256-column tile
// column), two of them (alternating by pass parity), then (256-aligned) the
// tile lists of the skipping shapes (TileLists, for at least 16 owned rows
// per tile).
size_t map_half_bytes(int rows, int cols);
int list_capacity(int rows, int cols);
size_t list_state_offset(int rows, int cols);
long long list_clear_u64(int rows, int cols);   // uint64 words cleared before a sequence
size_t change_map_bytes(int rows, int cols);
WsLayout ws_layout(const phgrms_params& p);

int hip_fail(hipError_t e, const char* what);
int validate_params(const phgrms_params& p);
int check_buffers(const uint8_t* d_in, const uint8_t* d_out, const phgrms_params& p,
                  const void* d_ws, size_t ws_bytes);
int size_class(long long npx);
int fused_shape(int beta, long long npx);
int set_grid_mode(int mode);
int grid_mode();
int set_fused_shape(int beta, int cls, int shape);   // cls -1: every class
// Shape of the batch path's multi-image launches (its own table: many
// images per launch favour other shapes than one image per launch).
int batch_shape(int beta, long long npx);
int set_batch_shape(int beta, int cls, int shape);   // cls -1: every class
TuneTables current_tuning();
void apply_tuning(const TuneTables& t);
// multi_pass_kernel<beta, shape> (batch.hip).
// maps: the kernel keeps change maps per image (tracking shapes only).
const void* multi_kernel_ptr(int beta, int shape, bool maps = false);
// Grid size for a pass kernel shape over `ntiles` tiles: one workgroup per
// tile, or at most the resident grid (CUs x resident workgroups) in grid
// mode 1.  persistent (a launch over listed tiles): kListedOversubscription
// resident grids, whatever the grid mode.  cycle: the launch runs the
// period-2 variant (its listed kernel's occupancy may differ).
int pass_grid(int beta, int shape, long long ntiles, bool persistent = false, bool cycle = false);
int enqueue_denoise(const uint8_t* d_in, uint8_t* d_out, const phgrms_params& p, int shape,
                    uint8_t* ws_img, unsigned long long* counts, unsigned long long* changed,
                    int* iterations, uint8_t* maps, hipStream_t s,
                    unsigned long long* diff2 = nullptr);

}  // namespace phg
