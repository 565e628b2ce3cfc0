// Pass pipelines of the N = 256 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(256)
