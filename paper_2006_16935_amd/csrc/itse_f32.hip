// FP32 storage and transforms (FP64 sums): kernel instantiations.
#include "itse_launch.h"

namespace itse {
template struct Launch<float>;
}
