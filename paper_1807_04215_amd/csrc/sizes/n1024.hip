// Pass pipelines of the N = 1024 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(1024)
