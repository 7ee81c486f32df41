// Ladder kernel variants and the autotuner's choice table.
//
// A variant is one kernel build able to run the batched ladder for a given
// n_nu and precision.  The table maps (precision, n_nu) to the variant the
// autotuner measured fastest; it lives for the process and, when the
// environment variable DF_TUNE_CACHE names a file, is read from and written to
// that file (one "prec n_nu name" line per entry).
#pragma once

namespace df {

enum LadderVariant {
    LV_GJB = 0,        // certified blocked Gauss-Jordan, FP64 MFMA, compiler's register budget
    LV_GJB_O3 = 1,     // same, capped for three waves per SIMD
    LV_VECTOR = 2,     // partial pivoting, FP64 vector FMAs
    LV_MFMA = 3,       // partial pivoting, FP64 MFMA trailing updates
    LV_MIXED = 4,      // certified FP32 sweep + FP64 residual correction
    LV_MIXED_O3 = 5,   // same, capped for three waves per SIMD
    LV_FP32 = 6,       // certified FP32 sweep alone
    LV_FP32_O4 = 7,    // same, capped for four waves per SIMD
    LV_FP32_O5 = 8,    // same, capped for five waves per SIMD
    LV_GJB_O4 = 9,     // certified FP64 kernel capped for four waves per SIMD (spills)
    LV_MIXED_O4 = 10,  // FP32 + FP64 refinement capped for four waves per SIMD (spills)
    LV_COUNT = 11
};

// A choice is a kernel variant and a launch shape: c = v + LV_COUNT * p, with
// p = 0 one work-group per item, p = 1, 2 a persistent grid of p times the
// resident work-groups, each taking items from its XCD's counter.  Its name is
// the variant's, with "@p1" / "@p2" appended for the persistent shapes.
constexpr int kPersistModes = 3;
constexpr int kChoices = LV_COUNT * kPersistModes;
inline int choice_variant(int c) { return c % LV_COUNT; }
inline int choice_persist(int c) { return c / LV_COUNT; }

const char *variant_name(int c);
int variant_from_name(const char *name);          // -1 if unknown
int variant_prec(int c);                            // precision class the variant delivers
bool variant_supports(int c, int n_nu, int prec);   // serves requests of this n_nu and precision
int variant_padded_size(int c, int n_nu);

// tuned choice for (prec, n_nu), or -1
int tuned_variant(int prec, int n_nu);
void set_tuned_variant(int prec, int n_nu, int c);
void clear_tuned();
int save_tune_cache();   // 0 on success or when no cache file is configured

}  // namespace df
