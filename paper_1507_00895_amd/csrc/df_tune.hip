// Autotuner choice table and its optional on-disk cache (host code).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <utility>

#include "../../include/df.h"
#include "df_internal.hpp"
#include "df_tune.hpp"

namespace df {

namespace {

const char *const kNames[LV_COUNT] = {"gjb",   "gjb_o3",   "vector",  "mfma",   "mixed",
                                     "mixed_o3", "fp32", "fp32_o4", "fp32_o5", "gjb_o4",
                                     "mixed_o4"};

std::mutex g_mu;
std::map<std::pair<int, int>, int> g_table;
bool g_loaded = false;

const char *cache_path() {
    const char *p = getenv("DF_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// caller holds g_mu
void load_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    int prec, n_nu;
    char name[32];
    while (fscanf(f, "%d %d %31s", &prec, &n_nu, name) == 3) {
        const int v = variant_from_name(name);
        if (v >= 0 && variant_supports(v, n_nu, prec)) g_table[{prec, n_nu}] = v;
    }
    fclose(f);
}

}  // namespace

const char *variant_name(int v) { return (v >= 0 && v < LV_COUNT) ? kNames[v] : "none"; }

int variant_from_name(const char *name) {
    if (!name) return -1;
    for (int v = 0; v < LV_COUNT; ++v)
        if (strcmp(name, kNames[v]) == 0) return v;
    return -1;
}

int variant_padded_size(int v, int n_nu) {
    switch (v) {
        case LV_GJB: return ladder_gjb_padded_size(n_nu);
        case LV_GJB_O3:
        case LV_GJB_O4: return ladder_gjb_has_occ3(n_nu) ? ladder_gjb_padded_size(n_nu) : 0;
        case LV_VECTOR: return ladder_padded_size(n_nu);
        case LV_MFMA: return ladder_mfma_padded_size(n_nu);
        case LV_MIXED: return ladder_mixed_padded_size(n_nu);
        case LV_MIXED_O3:
        case LV_MIXED_O4: return ladder_mixed_has_occ3(n_nu) ? ladder_mixed_padded_size(n_nu) : 0;
        case LV_FP32: return ladder_fp32_padded_size(n_nu);
        case LV_FP32_O4:
        case LV_FP32_O5: return ladder_mixed_padded_size(n_nu);
        default: return 0;
    }
}

int variant_prec(int v) {
    switch (v) {
        case LV_MIXED:
        case LV_MIXED_O3:
        case LV_MIXED_O4: return DF_FP32_REFINE;
        case LV_FP32:
        case LV_FP32_O4:
        case LV_FP32_O5: return DF_FP32;
        default: return DF_FP64;
    }
}

// A request is served by the variants of its own precision class; where that
// class has no kernel for n_nu (the refined kernels stop at n_nu = 64, the
// FP32 ones at 128), by the FP64 variants.
bool variant_supports(int v, int n_nu, int prec) {
    if (variant_padded_size(v, n_nu) == 0) return false;
    const int vp = variant_prec(v);
    if (vp == prec) return true;
    const int own = prec == DF_FP32 ? ladder_fp32_padded_size(n_nu) : ladder_mixed_padded_size(n_nu);
    return vp == DF_FP64 && prec != DF_FP64 && own == 0;
}

int tuned_variant(int prec, int n_nu) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_table.find({prec, n_nu});
    return it == g_table.end() ? -1 : it->second;
}

void set_tuned_variant(int prec, int n_nu, int v) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_table[{prec, n_nu}] = v;
}

void clear_tuned() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    g_loaded = true;   // a reset also forgets the cache file for this process
}

int save_tune_cache() {
    std::lock_guard<std::mutex> lk(g_mu);
    const char *path = cache_path();
    if (!path) return 0;
    FILE *f = fopen(path, "w");
    if (!f) return -1;
    for (const auto &e : g_table)
        fprintf(f, "%d %d %s\n", e.first.first, e.first.second, variant_name(e.second));
    return fclose(f) == 0 ? 0 : -1;
}

}  // namespace df
