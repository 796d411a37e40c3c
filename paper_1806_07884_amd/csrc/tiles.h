// Assembly of B by point tiles (tile_kernels.hip).
#pragma once

#include "plan_kernels.h"

namespace rbf {

// Points of one tile: a hash cell's points in sorted order, cut into pieces
// of at most this many.
constexpr int kTilePts = 512;

// Most centres a tile's window may hold (centres whose support can reach
// the tile's points), by dimension.
constexpr int tile_window_max(int dim) { return dim == 2 ? 256 : 384; }

// Per cell c < ncell: the number of tiles of its points (cnt[c]) and, for a
// cell that holds points, its window size (wcnt[c]: the active centres whose
// ball reaches the cell, widened by 1e-6 of a cell; 0 for an empty cell),
// atomically maxed into *maxwin; cnt[ncell] = wcnt[ncell] = 0.
hipError_t launch_tile_count(const PlanView& P, double cell_size, uint32_t* cnt, uint32_t* wcnt,
                             int32_t* maxwin, hipStream_t s);
// tiles[t] = {first point, end point, window offset, window size} (sorted
// point positions; the window's caller indices in wids), in cell order, from
// the exclusive scans off of cnt and woff of wcnt.
hipError_t launch_tile_fill(const PlanView& P, double cell_size, const uint32_t* off,
                            const uint32_t* woff, int4* tiles, int32_t* wids, hipStream_t s);
// The tiles' shares of B summed into acc (one uint64 per stored entry of the
// full pattern, zeroed by the caller; a pair's shares go to the entry in the
// row of its first window centre), in units of 2^(k - 63) with
// k = ceil((kexp[j] + kexp[l]) / 2) (kexp from launch_rhs): one block per
// tile.  Sets bit 1 of *err when a window exceeds tile_window_max (an
// internal error: the host checks the bound from launch_tile_count first).
hipError_t launch_tile_assemble(const PlanView& P, int phi, bool fp32, const int4* tiles,
                                int64_t ntiles, const int32_t* wids, const int64_t* row_ptr,
                                const int32_t* col, const int32_t* kexp,
                                unsigned long long* acc, int32_t* err, hipStream_t s);
// Each upper entry's value (its accumulator plus its mirror's) into the
// solver layout, upper entry and mirror, as T; and diag (0 for inactive
// centres).
hipError_t launch_tile_finish(const PlanView& P, bool fp32, const int64_t* row_ptr,
                              const int32_t* lower_cnt, const int32_t* col,
                              const int32_t* kexp, const unsigned long long* acc,
                              const int64_t* sptr, int lanes, void* val, double* diag,
                              hipStream_t s);

// ---- the pattern by point tiles
// Rows of cells in a centre's walk at radius 2 (5 in 2D, 25 in 3D).
int walk_rows(int dim);
// tab[c * (walk_rows + 1) + k] = {first sorted centre of row k of cell c's
// walk, the row's offset in the walk}, and at k = walk_rows {0, the walk's
// length}; the longest walk of a cell holding a centre maxed into *maxwalk.
hipError_t launch_walk_tables(const PlanView& P, int2* tab, int32_t* maxwalk, hipStream_t s);
// spos[l] = sorted position of centre l, ccell[l] = its cell id.
hipError_t launch_centre_slots(const PlanView& P, int32_t* spos, int32_t* ccell, hipStream_t s);
// Mark bits (words per row, zeroed by the caller) of every pair of window
// centres with a common point in some tile, at the column's position in the
// row's walk, both ways.  Bit 1 of *err: a window exceeds tile_window_max;
// bit 2: a mark position outside its row (never written; both internal
// errors).
// The marks of one tile gather in LDS first (max_nw * words words, max_nw
// the plan's widest window; the caller keeps that within
// tile_pattern_lds_max bytes) and go out with one atomic OR per nonzero word.
hipError_t launch_tile_pattern(const PlanView& P, const int4* tiles, int64_t ntiles,
                               const int32_t* wids, const int2* tab, const int32_t* spos,
                               const int32_t* ccell, int words, int max_nw, uint32_t* marks,
                               int32_t* err, hipStream_t s);
// Most bytes of a tile's LDS marks, by dimension (with the kernel's own LDS
// this keeps one workgroup per CU possible).
constexpr size_t tile_pattern_lds_max(int dim) { return dim == 2 ? 48 * 1024 : 64 * 1024; }
// From the marks: count mode writes full_cnt, lower_cnt (0 for inactive
// centres) and maxes the largest |l - j| into *maxdelta; fill mode writes
// each row's columns in ascending order at row_ptr.  Sets *err to 1 when a
// row exceeds kMaxCand entries.
hipError_t launch_mark_rows(const PlanView& P, bool fill, const int2* tab, const int32_t* ccell,
                            int words, const uint32_t* marks, int64_t* full_cnt,
                            int32_t* lower_cnt, const int64_t* row_ptr, int32_t* col,
                            int32_t* err, int32_t* maxdelta, hipStream_t s);

}  // namespace rbf
