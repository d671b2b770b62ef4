// The one-degree batched DG kernels with half the cells per block (tile
// variant 1 of the autotuner).
#define HPMG_TILE 1
#include "batch_dg_body.hpp"
