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

const char *variant_name(int c) {
    // "name", "name@p1", "name@p2" for every variant, built once
    static char names[kChoices][24];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int k = 0; k < kChoices; ++k) {
            const int v = choice_variant(k), p = choice_persist(k);
            if (p == 0) snprintf(names[k], sizeof names[k], "%s", kNames[v]);
            else snprintf(names[k], sizeof names[k], "%s@p%d", kNames[v], p);
        }
    });
    return (c >= 0 && c < kChoices) ? names[c] : "none";
}

int variant_from_name(const char *name) {
    if (!name) return -1;
    for (int c = 0; c < kChoices; ++c)
        if (strcmp(name, variant_name(c)) == 0) return c;
    return -1;
}

int variant_padded_size(int c, int n_nu) {
    if (c < 0 || c >= kChoices) return 0;
    const int v = choice_variant(c);
    // persistent grids: the FP64 certified builds with an item loop
    if (choice_persist(c) != 0 && v != LV_GJB && v != LV_GJB_O3) return 0;
    switch (v) {
        case LV_GJB: return ladder_gjb_padded_size(n_nu);
        case LV_GJB_O3:
        case LV_GJB_O4: return ladder_gjb_has_occ3(n_nu) ? ladder_gjb_padded_size(n_nu) : 0;
        case LV_VECTOR: return ladder_padded_size(n_nu);
        case LV_MFMA: return ladder_mfma_padded_size(n_nu);
        case LV_MIXED: return ladder_mixed_has_occ(n_nu, 0) ? ladder_mixed_padded_size(n_nu) : 0;
        case LV_MIXED_O3: return ladder_mixed_has_occ(n_nu, 3) ? ladder_mixed_padded_size(n_nu) : 0;
        case LV_MIXED_O4: return ladder_mixed_has_occ(n_nu, 4) ? ladder_mixed_padded_size(n_nu) : 0;
        case LV_FP32: return ladder_fp32_has_occ(n_nu, 0) ? ladder_fp32_padded_size(n_nu) : 0;
        case LV_FP32_O4: return ladder_fp32_has_occ(n_nu, 4) ? ladder_fp32_padded_size(n_nu) : 0;
        case LV_FP32_O5: return ladder_fp32_has_occ(n_nu, 5) ? ladder_fp32_padded_size(n_nu) : 0;
        default: return 0;
    }
}

int variant_prec(int c) {
    switch (choice_variant(c)) {
        case LV_MIXED:
        case LV_MIXED_O3:
        case LV_MIXED_O4: return DF_FP32_REFINE;
        case LV_FP32:
        case LV_FP32_O4:
        case LV_FP32_O5: return DF_FP32;
        default: return DF_FP64;
    }
}

// A request is served by the variants of its own precision class only (each
// class has kernels for every n_nu <= 128).
bool variant_supports(int c, int n_nu, int prec) {
    return variant_padded_size(c, n_nu) != 0 && variant_prec(c) == prec;
}

int tuned_variant(int prec, int n_nu) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_table.find({prec, n_nu});
    return it == g_table.end() ? -1 : it->second;
}

void set_tuned_variant(int prec, int n_nu, int c) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_table[{prec, n_nu}] = c;
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
