// Pass pipelines of the N = 768 grid, both precisions.
#include "../pipeline.hpp"

GRIDSPT_INSTANTIATE(768)
