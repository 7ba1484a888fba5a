// FP64 storage, transforms and sums: kernel instantiations.
#include "itse_launch.h"

namespace itse {
template struct Launch<double>;
}
