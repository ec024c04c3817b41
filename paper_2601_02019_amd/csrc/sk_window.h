// sk_window.h -- sliding-window sketches (Algorithm "ML-AeroSketch") behind
// the same C ABI.  Implemented in sk_window.cpp.
#pragma once
#include <stdint.h>

#include "../../include/sketch.h"

struct WindowState;

sk_status window_create(sketch_t h);
sk_status window_update(sketch_t h, const char* rows_dev, int64_t n, int64_t ld, int dtype);
sk_status window_query(sketch_t h, const double** out_f64);
// ATTP sketches: the sketch of the first t rows.
sk_status window_query_at(sketch_t h, int64_t t, const double** out_f64);
sk_status window_advance_impl(sketch_t h, int64_t t_now);
void window_destroy(sketch_t h);
const int32_t* window_info_ptr(sketch_t h);
int64_t window_time(sketch_t h);
int32_t window_levels(sketch_t h);
sk_status window_level_stats(sketch_t h, int32_t level, int64_t* st);
// P5 sketches (Algorithm "P5"): sites[e] in [0, m) checked by the caller.
sk_status p5_update_impl(sketch_t h, const int32_t* sites, const char* rows_dev, int64_t n, int64_t ld, int dtype);
void p5_counters(sketch_t h, int64_t* st8);
sk_status p5_coordinator_impl(sketch_t h, double* fhat, void* gram, int on_device);
// AeroSketchCOD sketches (sk_cod.cpp): device pointers, shapes checked by the caller.
sk_status cod_create(sketch_t h);
void cod_destroy(sketch_t h);
sk_status cod_update_impl(sketch_t h, const char* X, int64_t ldx, const char* Y, int64_t ldy, int64_t n, int dtype);
// A* (d x ell) and B* (d_y x ell), FP64 device buffers owned by the sketch.
sk_status cod_query_impl(sketch_t h, const double** A, const double** B);
// M_W (d x d_y, FP64) into device memory.
sk_status cod_product_impl(sketch_t h, double* M_dev);
void cod_stats(sketch_t h, int64_t* st6);
int64_t cod_time(sketch_t h);
const int32_t* cod_info_ptr(sketch_t h);
