// Work-list schedule kernels for C128 coupling tables (queue_kernels.h).
#include "queue_kernels.h"

namespace mqct {

const QKernelSet* queue_kernels_c128() {
  static QKernelSet table[QUEUE_SHAPES];
  static const bool filled = (queue::fill_all<C128, 0>(table), true);
  (void)filled;
  return table;
}

}  // namespace mqct
