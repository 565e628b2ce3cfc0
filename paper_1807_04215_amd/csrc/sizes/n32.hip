// Pass pipelines of the N = 32 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(32)
