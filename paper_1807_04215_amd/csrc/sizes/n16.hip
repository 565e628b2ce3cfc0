// Pass pipelines of the N = 16 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(16)
