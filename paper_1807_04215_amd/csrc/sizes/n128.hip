// Pass pipelines of the N = 128 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(128)
