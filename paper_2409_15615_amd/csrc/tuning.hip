// Process-wide launch tuning (kmg_set_tuning / kmg_get_tuning): the launch
// sites read it when they enqueue, so a captured graph keeps the shapes in
// force at capture time.
#include "kmg_internal.h"

namespace kmg {

namespace {
Tuning g_tuning;
}

const Tuning& tuning() { return g_tuning; }

bool set_tuning(const Tuning& t) {
    if (t.search_waves != 2 && t.search_waves != 4 && t.search_waves != 8) return false;
    if (t.count_queries != 1 && t.count_queries != 2 && t.count_queries != 4) return false;
    if (t.spfh_pair_mean < 0 || t.spfh_pair_mean > kMaxDegree) return false;
    if (t.fpfh_rows != 1 && t.fpfh_rows != 2 && t.fpfh_rows != 4 && t.fpfh_rows != 8 && t.fpfh_rows != 16)
        return false;
    if (t.band_tile != 0 && !band_tile_candidate(t.band_tile)) return false;
    if (t.fuse_features != 0 && t.fuse_features != 1) return false;
    if (t.xcd_split < 0 || t.xcd_split > 3) return false;
    if (t.match_form != 0 && t.match_form != 1) return false;
    if (t.search_form != 0 && t.search_form != 1) return false;
    g_tuning = t;
    return true;
}

}  // namespace kmg

extern "C" {

__attribute__((visibility("default"))) kmg_status kmg_set_tuning(const kmg_tuning* t) {
    kmg::Tuning v;  // defaults
    if (t) {
        v.search_waves = t->search_waves;
        v.count_queries = t->count_queries;
        v.spfh_pair_mean = t->spfh_pair_mean;
        v.fpfh_rows = t->fpfh_rows;
        v.band_tile = t->band_tile;
        v.fuse_features = t->fuse_features;
        v.xcd_split = t->xcd_split;
        v.match_form = t->match_form;
        v.search_form = t->search_form;
    }
    return kmg::set_tuning(v) ? KMG_OK : KMG_ERR_ARG;
}

__attribute__((visibility("default"))) kmg_status kmg_get_tuning(kmg_tuning* t) {
    if (!t) return KMG_ERR_ARG;
    const kmg::Tuning& v = kmg::tuning();
    t->search_waves = v.search_waves;
    t->count_queries = v.count_queries;
    t->spfh_pair_mean = v.spfh_pair_mean;
    t->fpfh_rows = v.fpfh_rows;
    t->band_tile = v.band_tile;
    t->fuse_features = v.fuse_features;
    t->xcd_split = v.xcd_split;
    t->match_form = v.match_form;
    t->search_form = v.search_form;
    return KMG_OK;
}

}  // extern "C"
