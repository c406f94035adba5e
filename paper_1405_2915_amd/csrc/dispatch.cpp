#include "dispatch.hpp"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

namespace skel {

int overlap2d_dense_variant(int64_t n, int radius) {
    return radius <= 2 && n >= (INT64_C(1) << 20) ? O2E_MARCH : O2B_LDS_TILE;
}

int overlap2d_separable_variant(int64_t n, int radius) {
    return radius <= 2 && n >= (INT64_C(1) << 20) ? O2E_MARCH : O2D_SEPARABLE_L1;
}

namespace {

const char* const kMap[] = {"M0_scalar", "M1_vec4", "M2_vec4x4_nt"};
const char* const kReduce[] = {"R0_single_wg", "R1_two_pass", "R2_ticket",
                               "R3_atomic", "R4_compensated", "R5_pairwise",
                               "R6_gather"};
const char* const kMapReduce[] = {"MR0_unfused", "MR1_fused_two_pass",
                                  "MR2_fused_ticket", "MR3_fused_single_wg",
                                  "MR4_compensated", "MR5_pairwise",
                                  "MR6_fused_gather"};
const char* const kOverlap1D[] = {"O1a_direct", "O1b_lds_tile", "O1c_shuffle"};
const char* const kOverlap2D[] = {"O2a_direct", "O2b_lds_tile", "O2c_lds_separable",
                                  "O2d_separable_l1", "O2e_march"};
const char* const kScan[] = {"S0_single_wg", "S1_reduce_then_scan",
                             "S2_decoupled_lookback", "S3_persistent_lookback",
                             "S4_small_tile_lookback", "S5_flat_lookback"};

const char* const kSegments[] = {"B0_per_segment", "B1_persistent"};
const char* const kScanRows[] = {"SR0_per_row", "SR1_wave_per_row"};
const char* const kAdjoint[] = {"A0_gather", "A1_flipped_forward"};
const char* const kChain[] = {"C0_composed", "C1_fused"};

const char* const kSkeletonNames[] = {"MAP",          "REDUCE", "MAPREDUCE",
                                      "MAPOVERLAP1D", "MAPOVERLAP2D", "SCAN",
                                      "REDUCE_SEGMENTS", "MAPOVERLAP1D_BACKWARD",
                                      "MAPOVERLAP2D_BACKWARD", "SCAN_ROWS",
                                      "MAP_OVERLAP2D_REDUCE"};
static_assert(sizeof kSkeletonNames / sizeof kSkeletonNames[0] == SKEL_SK_COUNT,
              "one name per skeleton id");
#define SKEL_NAMES_MATCH(table, count) \
    static_assert(sizeof table / sizeof table[0] == count, "one name per variant of " #table)
SKEL_NAMES_MATCH(kMap, MAP_NVAR);
SKEL_NAMES_MATCH(kReduce, REDUCE_NVAR);
SKEL_NAMES_MATCH(kMapReduce, MAPREDUCE_NVAR);
SKEL_NAMES_MATCH(kOverlap1D, OVERLAP1D_NVAR);
SKEL_NAMES_MATCH(kOverlap2D, OVERLAP2D_NVAR);
SKEL_NAMES_MATCH(kScan, SCAN_NVAR);
SKEL_NAMES_MATCH(kSegments, SEGMENTS_NVAR);
SKEL_NAMES_MATCH(kScanRows, SCANROWS_NVAR);
SKEL_NAMES_MATCH(kAdjoint, ADJOINT_NVAR);
SKEL_NAMES_MATCH(kChain, CHAIN_NVAR);
#undef SKEL_NAMES_MATCH

struct TableEntry {
    int skeleton;
    int dtype;
    int log2n;
    int variant;
    int cls;  // stencil class the entry was tuned on (stencil skeletons), else -1
};

bool is_stencil(int skeleton) {
    return skeleton == SKEL_SK_MAPOVERLAP1D || skeleton == SKEL_SK_MAPOVERLAP2D ||
           skeleton == SKEL_SK_MAPOVERLAP1D_BACKWARD || skeleton == SKEL_SK_MAPOVERLAP2D_BACKWARD;
}

// The stencil class of a call: the radius in 1D; separable + 2 * max(ry, rx)
// in 2D (the encoding of skel_select_variant's aux).  Variants rank
// differently for different radii and weight forms, so a table entry applies
// only to calls of the class it was tuned on.
int stencil_class(const CallContext& c) {
    if (c.skeleton == SKEL_SK_MAPOVERLAP1D || c.skeleton == SKEL_SK_MAPOVERLAP1D_BACKWARD)
        return c.radius;
    if (c.skeleton == SKEL_SK_MAPOVERLAP2D || c.skeleton == SKEL_SK_MAPOVERLAP2D_BACKWARD)
        return c.separable + 2 * c.radius;
    return -1;
}
std::vector<TableEntry> g_table;
std::mutex g_table_mu;

int ceil_log2(int64_t n) {
    int k = 0;
    while (k < 62 && (INT64_C(1) << k) < n) ++k;
    return k;
}

int find_variant(int skeleton, const char* name) {
    int nv = variant_count(skeleton);
    for (int v = 0; v < nv; ++v)
        if (std::strcmp(variant_name(skeleton, v), name) == 0) return v;
    char* end = nullptr;
    long k = std::strtol(name, &end, 10);
    if (end && *end == '\0' && end != name && k >= 0 && k < nv) return (int)k;
    return -1;
}

int static_rule(const CallContext& c) {
    switch (c.skeleton) {
    case SKEL_SK_MAP: return c.n < (INT64_C(1) << 14) ? M1_VEC4 : M2_VEC4X4_NT;
    // (the tuned binary32 plan's choices, for the types it does not cover: one
    // workgroup for small arrays, then the ticket-free gather)
    case SKEL_SK_REDUCE: return c.n <= (INT64_C(1) << 15) ? R0_SINGLE_WG : R6_GATHER;
    case SKEL_SK_MAPREDUCE:
        return c.n <= (INT64_C(1) << 15) ? MR3_FUSED_SINGLE_WG : MR6_FUSED_GATHER;
    case SKEL_SK_MAPOVERLAP1D:
        // up to 2^20 elements the direct form (its loads hit the cache; as the
        // tuned plan has it for radius 2), beyond that the cross-lane form
        if (c.radius > 4) return O1B_LDS_TILE;
        return c.n <= (INT64_C(1) << 20) ? O1A_DIRECT : O1C_SHUFFLE;
    case SKEL_SK_MAPOVERLAP2D:
        return c.separable ? overlap2d_separable_variant(c.n, c.radius)
                           : overlap2d_dense_variant(c.n, c.radius);
    case SKEL_SK_SCAN:
        // the flat look-back while the array fits its 1024 tiles (the tuned plan's
        // choice for int32 up to 2^22, and its binary32 combination order is
        // fixed, so float scans are bit-stable run to run); beyond, the persistent
        // look-back
        return c.n <= kFlatMaxTiles * scan_flat_tile(c.din) ? S5_FLAT_LOOKBACK
                                                            : S3_PERSISTENT_LOOKBACK;
    case SKEL_SK_REDUCE_SEGMENTS: return B1_PERSISTENT;
    case SKEL_SK_SCAN_ROWS:
        // a few long rows: one single-pass scan per row fills the device;
        // otherwise one wavefront per row
        return c.rows_aligned && c.rows < 64 && c.cols >= (INT64_C(1) << 20) ? SR0_PER_ROW
                                                                              : SR1_WAVE_PER_ROW;
    case SKEL_SK_MAPOVERLAP1D_BACKWARD:
    case SKEL_SK_MAPOVERLAP2D_BACKWARD: return A1_FLIPPED_FORWARD;
    case SKEL_SK_MAP_OVERLAP2D_REDUCE: return C1_FUSED;
    }
    return -1;
}

int table_rule(const CallContext& c) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    if (g_table.empty()) return -1;
    int key = ceil_log2(c.n < 1 ? 1 : c.n);
    const int cls = stencil_class(c);
    int best = -1, best_k = -1, lowest = -1, lowest_k = 1 << 30;
    for (const auto& e : g_table) {
        if (e.skeleton != c.skeleton || e.dtype != (int)c.din || e.cls != cls) continue;
        if (e.log2n <= key && e.log2n > best_k) {
            best = e.variant;
            best_k = e.log2n;
        }
        if (e.log2n < lowest_k) {
            lowest = e.variant;
            lowest_k = e.log2n;
        }
    }
    return best >= 0 ? best : lowest;  // below the table: its smallest size
}

bool log_enabled() {
    const char* s = std::getenv("SKEL_LOG");
    return s && *s && std::strcmp(s, "0") != 0;
}

}  // namespace

int variant_count(int skeleton) {
    switch (skeleton) {
    case SKEL_SK_MAP: return MAP_NVAR;
    case SKEL_SK_REDUCE: return REDUCE_NVAR;
    case SKEL_SK_MAPREDUCE: return MAPREDUCE_NVAR;
    case SKEL_SK_MAPOVERLAP1D: return OVERLAP1D_NVAR;
    case SKEL_SK_MAPOVERLAP2D: return OVERLAP2D_NVAR;
    case SKEL_SK_SCAN: return SCAN_NVAR;
    case SKEL_SK_REDUCE_SEGMENTS: return SEGMENTS_NVAR;
    case SKEL_SK_SCAN_ROWS: return SCANROWS_NVAR;
    case SKEL_SK_MAPOVERLAP1D_BACKWARD:
    case SKEL_SK_MAPOVERLAP2D_BACKWARD: return ADJOINT_NVAR;
    case SKEL_SK_MAP_OVERLAP2D_REDUCE: return CHAIN_NVAR;
    }
    return 0;
}

const char* variant_name(int skeleton, int v) {
    if (v < 0 || v >= variant_count(skeleton)) return nullptr;
    switch (skeleton) {
    case SKEL_SK_MAP: return kMap[v];
    case SKEL_SK_REDUCE: return kReduce[v];
    case SKEL_SK_MAPREDUCE: return kMapReduce[v];
    case SKEL_SK_MAPOVERLAP1D: return kOverlap1D[v];
    case SKEL_SK_MAPOVERLAP2D: return kOverlap2D[v];
    case SKEL_SK_SCAN: return kScan[v];
    case SKEL_SK_REDUCE_SEGMENTS: return kSegments[v];
    case SKEL_SK_SCAN_ROWS: return kScanRows[v];
    case SKEL_SK_MAPOVERLAP1D_BACKWARD:
    case SKEL_SK_MAPOVERLAP2D_BACKWARD: return kAdjoint[v];
    case SKEL_SK_MAP_OVERLAP2D_REDUCE: return kChain[v];
    }
    return nullptr;
}

bool selectable(int v, const CallContext& c, const char** why) {
    static const char* ok = "";
    const char* dummy;
    if (!why) why = &dummy;
    *why = ok;
    if (v < 0 || v >= variant_count(c.skeleton)) {
        *why = "no such variant";
        return false;
    }
    switch (c.skeleton) {
    case SKEL_SK_REDUCE:
        // hardware float atomics give sums only; integer min/max atomics exist
        if (v == R3_ATOMIC && c.op != SKEL_SUM &&
            (c.din == SKEL_F32 || c.din == SKEL_BF16)) {
            *why = "atomic finish supports floating-point SUM only";
            return false;
        }
        if ((v == R4_COMPENSATED || v == R5_PAIRWISE) &&
            (c.op != SKEL_SUM || (c.din != SKEL_F32 && c.din != SKEL_BF16))) {
            *why = "compensated and pairwise summation apply to floating-point SUM only";
            return false;
        }
        return true;
    case SKEL_SK_MAPREDUCE:
        // the unfused form stores the mapped values with the F32 Map skeleton
        if (v == MR0_UNFUSED && c.din != SKEL_F32) {
            *why = "unfused form needs F32 inputs (Map is F32)";
            return false;
        }
        if ((v == MR4_COMPENSATED || v == MR5_PAIRWISE) && c.op != SKEL_SUM) {
            *why = "compensated and pairwise summation apply to SUM only";
            return false;
        }
        return true;
    case SKEL_SK_MAPOVERLAP1D:
        if (v == O1C_SHUFFLE && c.radius > 4) {
            *why = "cross-lane variant reaches at most 4 neighbours per side";
            return false;
        }
        return true;
    case SKEL_SK_MAPOVERLAP2D:
        if ((v == O2C_LDS_SEPARABLE || v == O2D_SEPARABLE_L1) && !c.separable) {
            *why = "separable variants need the weights as factors wy, wx";
            return false;
        }
        if (v == O2E_MARCH && c.radius > 4) {
            *why = "marching variant reaches at most 4 neighbours per side";
            return false;
        }
        return true;
    case SKEL_SK_SCAN:
        if (c.reverse && v != S2_LOOKBACK && v != S3_PERSISTENT_LOOKBACK &&
            v != S4_SMALL_TILE_LOOKBACK && v != S5_FLAT_LOOKBACK) {
            *why = "reverse scans run in the single-pass variants only";
            return false;
        }
        if (v == S5_FLAT_LOOKBACK && c.n > kFlatMaxTiles * scan_flat_tile(c.din)) {
            *why = "flat look-back takes at most 1024 tiles (2^22 elements, 2^21 for I64)";
            return false;
        }
        return true;
    case SKEL_SK_SCAN_ROWS:
        if (v == SR0_PER_ROW && !c.rows_aligned) {
            *why = "per-row single-pass scans need 16-byte aligned row starts";
            return false;
        }
        return true;
    default: return true;
    }
}

int choose_variant(int requested, const CallContext& c, skel_status* st) {
    *st = SKEL_OK;
    const char* why = "";
    int v = -1;
    const char* source = "forced";
    if (requested != SKEL_VARIANT_AUTO) {
        if (!selectable(requested, c, &why)) {
            *st = fail(SKEL_E_UNSUPPORTED, "%s variant %d (%s) not selectable: %s",
                       kSkeletonNames[c.skeleton], requested,
                       variant_name(c.skeleton, requested)
                           ? variant_name(c.skeleton, requested)
                           : "?",
                       why);
            return -1;
        }
        v = requested;
    } else {
        char key[64];
        std::snprintf(key, sizeof key, "SKEL_VARIANT_%s", kSkeletonNames[c.skeleton]);
        const char* env = std::getenv(key);
        if (env && *env) {
            v = find_variant(c.skeleton, env);
            source = "environment";
            if (v < 0 || !selectable(v, c, &why)) v = -1;
        }
        if (v < 0) {
            v = table_rule(c);
            source = "table";
            if (v >= 0 && !selectable(v, c, &why)) v = -1;
        }
        if (v < 0) {
            v = static_rule(c);
            source = "static";
        }
        if (v < 0 || !selectable(v, c, &why)) {
            *st = fail(SKEL_E_UNSUPPORTED, "no selectable %s variant",
                       kSkeletonNames[c.skeleton]);
            return -1;
        }
    }
    if (log_enabled())
        std::fprintf(stderr, "[skel] %s n=%lld dtype=%s -> %s (%s)\n",
                     kSkeletonNames[c.skeleton], (long long)c.n, dtype_name(c.din),
                     variant_name(c.skeleton, v), source);
    return v;
}

skel_status load_plan_table(const char* path) {
    if (!path) return fail(SKEL_E_INVAL, "null path");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(SKEL_E_INVAL, "cannot open plan table %s", path);
    std::vector<TableEntry> t;
    char line[256];
    int lineno = 0;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        char* p = line;
        while (std::isspace((unsigned char)*p)) ++p;
        if (*p == '#' || *p == '\0') continue;
        char sk[32], dt[16], vn[64];
        int lg, cls = -1;
        const int got = std::sscanf(p, "%31s %15s %d %63s %d", sk, dt, &lg, vn, &cls);
        if (got != 4 && got != 5) {
            std::fclose(f);
            return fail(SKEL_E_INVAL,
                        "%s:%d: expected <skeleton> <dtype> <log2n> <variant> [<class>]", path,
                        lineno);
        }
        int s = -1, d = -1;
        for (int k = 0; k < SKEL_SK_COUNT; ++k)
            if (std::strcmp(sk, kSkeletonNames[k]) == 0) s = k;
        for (int k = SKEL_F32; k <= SKEL_I64; ++k)
            if (std::strcmp(dt, dtype_name((skel_dtype)k)) == 0) d = k;
        int v = s >= 0 ? find_variant(s, vn) : -1;
        if (s < 0 || d < 0 || v < 0 || lg < 0 || lg > 62) {
            std::fclose(f);
            return fail(SKEL_E_INVAL, "%s:%d: unknown skeleton, dtype or variant", path,
                        lineno);
        }
        if (is_stencil(s) != (got == 5) || (got == 5 && cls < 0)) {
            std::fclose(f);
            return fail(SKEL_E_INVAL,
                        "%s:%d: MapOverlap entries carry the stencil class they were tuned on "
                        "(radius in 1D, separable + 2 * radius in 2D); other entries do not",
                        path, lineno);
        }
        t.push_back({s, d, lg, v, cls});
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_table_mu);
    g_table.swap(t);
    return SKEL_OK;
}

void clear_plan_table() {
    std::lock_guard<std::mutex> lk(g_table_mu);
    g_table.clear();
}

int plan_table_size() {
    std::lock_guard<std::mutex> lk(g_table_mu);
    return (int)g_table.size();
}

}  // namespace skel

extern "C" {

int skel_variant_count(int skeleton) { return skel::variant_count(skeleton); }

const char* skel_variant_name(int skeleton, int variant) {
    return skel::variant_name(skeleton, variant);
}

int skel_select_variant(int skeleton, skel_dtype dtype, int64_t n, int64_t rows,
                        int64_t cols, int aux) {
    if (skeleton < 0 || skeleton >= SKEL_SK_COUNT || !skel::dtype_valid(dtype)) return -1;
    skel::CallContext c;
    c.skeleton = skeleton;
    c.din = dtype;
    c.dout = dtype;
    c.n = n;
    c.rows = rows;
    c.cols = cols;
    if (skeleton == SKEL_SK_MAPOVERLAP1D || skeleton == SKEL_SK_MAPOVERLAP1D_BACKWARD)
        c.radius = aux;
    else if (skeleton == SKEL_SK_SCAN) c.reverse = aux;
    else if (skeleton == SKEL_SK_SCAN_ROWS) {
        c.reverse = aux;
        c.rows_aligned = skel::rows_aligned(dtype, dtype, cols);
    } else if (skeleton == SKEL_SK_MAPOVERLAP2D || skeleton == SKEL_SK_MAPOVERLAP2D_BACKWARD) {
        c.separable = aux & 1;
        c.radius = aux >> 1;
    }
    skel_status st;
    return skel::choose_variant(SKEL_VARIANT_AUTO, c, &st);
}

skel_status skel_load_plan(const char* path) { return skel::load_plan_table(path); }

skel_status skel_clear_plan(void) {
    skel::clear_plan_table();
    return SKEL_OK;
}

}  // extern "C"
