// Block one-sided Jacobi: placeholder driver until the block kernels land.
#include "../../include/jevd.h"
#include "block.h"

namespace jevd {

bool block_width_supported(int b) { return b == 16 || b == 32 || b == 64; }

bool block_shape_supported(int m, int n, int b)
{
    return block_width_supported(b) && n % (2 * b) == 0 && n >= 4 * b && m >= n;
}

int choose_block_width(int m, int n)
{
    (void)m;
    (void)n;
    return 32;
}

int auto_variant(int m, int n)
{
    (void)m;
    (void)n;
    return JEVD_VAR_POINTWISE;
}

int run_block(BlockWorkspace *ws, const BlockRunArgs &a, int *sweeps_done)
{
    (void)ws;
    (void)a;
    *sweeps_done = 0;
    return JEVD_EINVAL;
}

void block_workspace_free(BlockWorkspace *ws) { (void)ws; }

}  // namespace jevd
