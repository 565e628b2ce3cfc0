// Pass pipelines of the N = 64 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(64)
