// Pass pipelines of the N = 192 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(192)
