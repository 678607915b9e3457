// FP64 dense linear algebra for the low-rank step (placeholder).
#include "internal.hpp"
