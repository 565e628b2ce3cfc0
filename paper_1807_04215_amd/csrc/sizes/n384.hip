// Pass pipelines of the N = 384 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(384)
