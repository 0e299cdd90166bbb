// tuned_gfx950.h -- the library's built-in tuned tables for MI355X (gfx950).
// Written by build.py on every build from the autotuner's records
// (tuning/batch_gfx950.json, tuning/variants_gfx950.json); do not edit by hand:
// rerun paper_2307_16652_amd.tune, then the build.
#pragma once

#include <stdint.h>

#include "pald.h"

namespace pald_tuned {

// batched mode: per-size buckets (n_max ascending), persistent grid per CU
// (0 = resident capacity), queue lag (0 = default) and launch form
constexpr pald_batch_bucket kBatchBuckets[] = {
    {128, 64, 1, 0},
    {256, 64, 1, 0},
    {512, 64, 1, 0},
    {1073741824, 64, 1, 0}};
constexpr int32_t kBatchWorkgroupsPerCu = 0;
constexpr int32_t kBatchQueueLag = 0;
constexpr bool kBatchSplitPass1 = true;

// single-matrix variant for PALD_VARIANT_AUTO, with the pass-2 y split and
// the pass-1 z split it was fastest with (0 = the automatic split): the entry
// with the largest n not above the problem's n (the first entry below that)
struct VariantPick {
    int64_t n;
    int32_t variant;
    int32_t y_chunks;
    int32_t z_chunks;
};
constexpr VariantPick kVariants[] = {
    {256, PALD_VARIANT_PAIRWISE, 8, 0},
    {512, PALD_VARIANT_PAIRWISE, 8, 0},
    {1024, PALD_VARIANT_PAIRWISE, 8, 0},
    {2048, PALD_VARIANT_PAIRWISE, 8, 0},
    {4096, PALD_VARIANT_HYBRID2, 0, 1},
    {8192, PALD_VARIANT_HYBRID2, 0, 1},
    {16384, PALD_VARIANT_HYBRID2, 0, 0},
    {32768, PALD_VARIANT_HYBRID2, 0, 2}};

}  // namespace pald_tuned
