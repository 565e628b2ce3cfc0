// Pass pipelines of the N = 96 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(96)
