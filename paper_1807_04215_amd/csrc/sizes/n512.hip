// Pass pipelines of the N = 512 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(512)
