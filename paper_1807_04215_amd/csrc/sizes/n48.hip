// Pass pipelines of the N = 48 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(48)
