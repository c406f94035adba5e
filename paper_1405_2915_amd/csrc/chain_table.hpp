// Host side of the fused call chain Map -> MapOverlap 2D -> Reduce SUM: how
// often, weighted, the 2D neighbourhood map of a field reads each element
// (the column sums A^T 1 of the map), tabulated per row class x column class.
// Plain C++ (no HIP), so the table is also checked on the CPU.
#pragma once

#include <cstdint>

#include "skel.h"

namespace skel {

constexpr int kChainMaxClasses = 2 * SKEL_MAX_RADIUS_2D + 1;

// Rows (columns) within ry (rx) of a field's edge have classes of their own
// (0 .. r-1 from the first row, r+1 .. 2r up to the last); all others share
// class r, the interior.  A field with fewer than 2r + 1 rows (columns) gives
// every row (column) its own class.
struct ChainTable {
    int64_t rows, cols;
    int ry, rx;
    int small_r, small_c;  // fewer than 2r + 1 rows / columns
    int nrc, ncc;          // row and column classes
    float interior;        // the interior entry: the sum of the weights
    float tab[kChainMaxClasses * kChainMaxClasses];  // tab[rc * ncc + cc]
    double pad_total;      // sum of W[a][b] * pad over every pad read (CONST)
};

// Fill *t for `fields` fields of rows x cols (rows, cols >= 1), weights w2d
// ((2ry+1) x (2rx+1)) or the factors wy, wx, radii up to SKEL_MAX_RADIUS_2D.
void chain_table(int64_t rows, int64_t cols, int64_t fields, const float* w2d, const float* wy,
                 const float* wx, int ry, int rx, int edge, float pad, ChainTable* t);

// the class of field-local row r / column c
int chain_row_class(const ChainTable& t, int64_t r);
int chain_col_class(const ChainTable& t, int64_t c);

}  // namespace skel
