// sk_window.cpp -- placeholder until the window engine lands.
#include "sk_window.h"

sk_status window_create(sketch_t) { return SK_EUNSUPPORTED; }
sk_status window_update(sketch_t, const char*, int64_t, int64_t, int) { return SK_EUNSUPPORTED; }
sk_status window_query(sketch_t, const double**) { return SK_EUNSUPPORTED; }
sk_status window_advance_impl(sketch_t, int64_t) { return SK_EUNSUPPORTED; }
void window_destroy(sketch_t) {}
const int32_t* window_info_ptr(sketch_t) { return nullptr; }
int64_t window_time(sketch_t) { return 0; }
int32_t window_levels(sketch_t) { return 1; }
