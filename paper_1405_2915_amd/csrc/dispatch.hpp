// Variant registry and execution plan.
//
// Section III: each skeleton has several implementation variants, and an
// execution plan attached to the skeleton gives the expected best one for the
// current call context (problem size, ...).  Section II: conditional
// composition restricts which variants are selectable for a context, and the
// plan may come from static rules or from off-line tuning (a precomputed,
// size-keyed dispatch structure looked up at run time).
#pragma once

#include "common.hpp"

namespace skel {

// variant indices (stable: they are the values of the `variant` argument)
enum MapVariant { M0_SCALAR = 0, M1_VEC4 = 1, M2_VEC4X4_NT = 2, MAP_NVAR };
enum ReduceVariant { R0_SINGLE_WG = 0, R1_TWO_PASS = 1, R2_TICKET = 2, R3_ATOMIC = 3,
                     R4_COMPENSATED = 4, R5_PAIRWISE = 5, R6_GATHER = 6, REDUCE_NVAR };
enum MapReduceVariant { MR0_UNFUSED = 0, MR1_FUSED_TWO_PASS = 1, MR2_FUSED_TICKET = 2,
                        MR3_FUSED_SINGLE_WG = 3, MR4_COMPENSATED = 4, MR5_PAIRWISE = 5,
                        MR6_FUSED_GATHER = 6, MAPREDUCE_NVAR };
enum Overlap1DVariant { O1A_DIRECT = 0, O1B_LDS_TILE = 1, O1C_SHUFFLE = 2, OVERLAP1D_NVAR };
enum Overlap2DVariant { O2A_DIRECT = 0, O2B_LDS_TILE = 1, O2C_LDS_SEPARABLE = 2,
                        O2D_SEPARABLE_L1 = 3, O2E_MARCH = 4, OVERLAP2D_NVAR };
enum ScanVariant { S0_SINGLE_WG = 0, S1_REDUCE_THEN_SCAN = 1, S2_LOOKBACK = 2,
                   S3_PERSISTENT_LOOKBACK = 3, S4_SMALL_TILE_LOOKBACK = 4, S5_FLAT_LOOKBACK = 5,
                   SCAN_NVAR };
// S5 (flat look-back): elements per tile for an input type, and the most tiles
// one call may have (every tile reads all its predecessors' totals)
constexpr int64_t scan_flat_tile(int din) { return din == SKEL_I64 ? 2048 : 4096; }
constexpr int64_t kFlatMaxTiles = 1024;
enum SegmentsVariant { B0_PER_SEGMENT = 0, B1_PERSISTENT = 1, SEGMENTS_NVAR };
enum ScanRowsVariant { SR0_PER_ROW = 0, SR1_WAVE_PER_ROW = 1, SCANROWS_NVAR };
// the call chain Map -> MapOverlap 2D -> Reduce SUM (forward and backward)
enum ChainVariant { C0_COMPOSED = 0, C1_FUSED = 1, CHAIN_NVAR };
// MapOverlap adjoints (1D and 2D share the names)
enum AdjointVariant { A0_GATHER = 0, A1_FLIPPED_FORWARD = 1, ADJOINT_NVAR };

// What the plan may look at for one call.
struct CallContext {
    int skeleton = 0;
    skel_dtype din = SKEL_F32, dout = SKEL_F32;
    int64_t n = 0, rows = 0, cols = 0;
    int op = 0;         // reduce op (Reduce/MapReduce/Scan) or map op (Map)
    int map_op = 0;     // MapReduce's element function
    int separable = 0;  // MapOverlap2D: weights given as factors
    int radius = 0;     // MapOverlap1D radius; MapOverlap2D: max(ry, rx)
    int reverse = 0;    // Scan: a reverse (suffix) kind
    int rows_aligned = 0;  // row-wise Scan: every row starts 16-byte aligned
};

// 2D neighbourhood map with a dense (non-separable) weight matrix: the
// marching window for radii up to 2 on 2^20 elements or more, else the LDS
// tile.  Measured with the Infinity Cache evicted before each call, marching
// window against LDS tile: 5-point stencil on 64 fields of 2048^2 357 / 426
// us, on 16384^2 360 / 443, on 2048^2 8.6 / 13.0 (on 8192^2 96 / 84); 5 x 5
// on 16384^2 379 / 452.  Dense 9 x 9 loses (4096^2: 96 / 68 us; its 64-row
// strips or shorter ones).  Also the forward pass that the flipped transpose
// runs.
int overlap2d_dense_variant(int64_t n, int radius);
// The same with the weights given as factors: the marching window for radii up
// to 2 on 2^20 elements or more (3 x 3 over 64 fields of 2048^2: 357 against
// 388 us, caches evicted), else the separable L1 variant (the 9 x 9 Gaussian:
// level on 4096^2, slower for the marching window elsewhere).
int overlap2d_separable_variant(int64_t n, int radius);

int variant_count(int skeleton);
const char* variant_name(int skeleton, int variant);

// Selectability constraint of one variant for a context (conditional
// composition).  Returns true, or false and sets *why to a reason.
bool selectable(int variant, const CallContext& ctx, const char** why);

// The execution plan: forced variant (checked), an environment override
// SKEL_VARIANT_<SKELETON>=<name or index>, a loaded size-keyed table, or the
// static rules, in that order.  Returns the variant or a negative status.
int choose_variant(int requested, const CallContext& ctx, skel_status* st);

// Size-keyed dispatch table (off-line tuning result).  Text format, one entry
// per line:  <skeleton> <dtype> <log2 n> <variant name>
// Lookup takes the entry with the largest log2 n not above ceil(log2(n)) for
// the skeleton and dtype; sizes beyond the table extrapolate from the last.
skel_status load_plan_table(const char* path);
void clear_plan_table();
int plan_table_size();

}  // namespace skel
