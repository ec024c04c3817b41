// k_window.hip -- kernels of the sliding-window sketch (placeholder).
#include "sk_device.h"
