// The (A^T 1) table of the fused call chain (see chain_table.hpp).
#include "chain_table.hpp"

namespace skel {
namespace {

double weight_at(const float* w2d, const float* wy, const float* wx, int rx, int a, int b) {
    if (w2d) return (double)w2d[a * (2 * rx + 1) + b];
    return (double)wy[a] * (double)wx[b];
}

// read counts along one axis of length len: cnt[a] = #{p in [0, len) :
// e(p + a - r) = i}, the outputs whose tap a reads element i (pad reads
// count nowhere)
void axis_counts(int64_t i, int64_t len, int r, int edge, int* cnt) {
    for (int a = 0; a <= 2 * r; ++a) {
        int k = 0;
        if (edge == SKEL_EDGE_CYCLIC) {
            k = 1;  // p -> (p + a - r) mod len is a bijection of [0, len)
        } else {
            const int64_t p = i - a + r;  // the read that lands on i directly
            if (p >= 0 && p < len) k = 1;
            if (edge == SKEL_EDGE_CLAMP) {
                // reads past an end land on that end: p + a - r < 0 on element
                // 0, p + a - r > len - 1 on element len - 1 (both if len = 1)
                for (int64_t q = 0; q < len && q + a - r < 0; ++q)
                    if (i == 0) ++k;
                for (int64_t q = len - 1; q >= 0 && q + a - r > len - 1; --q)
                    if (i == len - 1) ++k;
            }
        }
        cnt[a] = k;
    }
}

// a row (column) of class c: c itself near the start, its mirror near the
// end, r for the interior class
int64_t class_member(int c, int r, int64_t len, int small) {
    if (small || c < r) return c;
    if (c > r) return len - 1 - (2 * r - c);
    return r;
}

}  // namespace

void chain_table(int64_t rows, int64_t cols, int64_t fields, const float* w2d, const float* wy,
                 const float* wx, int ry, int rx, int edge, float pad, ChainTable* t) {
    t->rows = rows;
    t->cols = cols;
    t->ry = ry;
    t->rx = rx;
    t->small_r = rows < 2 * ry + 1;
    t->small_c = cols < 2 * rx + 1;
    t->nrc = t->small_r ? (int)rows : 2 * ry + 1;
    t->ncc = t->small_c ? (int)cols : 2 * rx + 1;
    for (int k = 0; k < kChainMaxClasses * kChainMaxClasses; ++k) t->tab[k] = 0.0f;
    int cy[kChainMaxClasses], cx[kChainMaxClasses];
    for (int rc = 0; rc < t->nrc; ++rc) {
        axis_counts(class_member(rc, ry, rows, t->small_r), rows, ry, edge, cy);
        for (int cc = 0; cc < t->ncc; ++cc) {
            axis_counts(class_member(cc, rx, cols, t->small_c), cols, rx, edge, cx);
            double s = 0.0;
            for (int a = 0; a <= 2 * ry; ++a)
                for (int b = 0; b <= 2 * rx; ++b)
                    s += weight_at(w2d, wy, wx, rx, a, b) * (double)cy[a] * (double)cx[b];
            t->tab[rc * t->ncc + cc] = (float)s;
        }
    }
    t->interior = (!t->small_r && !t->small_c) ? t->tab[ry * t->ncc + rx] : 0.0f;
    // CONST borders: tap (a, b) reads inside the field for
    // (rows - |a - ry|) x (cols - |b - rx|) outputs and the pad for the rest
    double padsum = 0.0;
    if (edge == SKEL_EDGE_CONST && pad != 0.0f) {
        for (int a = 0; a <= 2 * ry; ++a)
            for (int b = 0; b <= 2 * rx; ++b) {
                const int64_t ny = rows - (a > ry ? a - ry : ry - a);
                const int64_t nx = cols - (b > rx ? b - rx : rx - b);
                const double inside = (double)(ny > 0 ? ny : 0) * (double)(nx > 0 ? nx : 0);
                padsum += weight_at(w2d, wy, wx, rx, a, b) * ((double)rows * (double)cols - inside);
            }
        padsum *= (double)pad * (double)fields;
    }
    t->pad_total = padsum;
}

int chain_row_class(const ChainTable& t, int64_t r) {
    if (t.small_r || r < t.ry) return (int)r;
    if (r >= t.rows - t.ry) return 2 * t.ry - (int)(t.rows - 1 - r);
    return t.ry;
}

int chain_col_class(const ChainTable& t, int64_t c) {
    if (t.small_c || c < t.rx) return (int)c;
    if (c >= t.cols - t.rx) return 2 * t.rx - (int)(t.cols - 1 - c);
    return t.rx;
}

}  // namespace skel
