// host_walk.hip -- TEST INFRASTRUCTURE: the two-step kernel's strip walk and
// its multiply-and-shift divisions (strip_walk, fast_div, div_by,
// strip_tile of the kernels' headers) compiled for the host, so that a CPU
// test can hold them against integer division and the plain strip walk.
// Built by tests/test_step2_cpu.py with hipcc --offload-host-only; never part
// of the library.
#include "clbm_step2.h"

extern "C" {
// n / d as the kernels divide (0 <= n < 2^31, d >= 1).
int host_div_by(uint32_t d, int n) { return clbm::div_by(n, clbm::fast_div(d)); }

// Tile (tx[t], ty[t]) of every t < count in the walk of a tiles_x x tiles_y
// lattice in strips of sw tile columns.
void host_strip_walk(int tiles_x, int tiles_y, int sw, const int *t, int count, int *tx, int *ty)
{
    const clbm::StripWalk p = clbm::strip_walk(tiles_x, tiles_y, sw);
    for (int k = 0; k < count; ++k) clbm::strip_tile(t[k], p, tx[k], ty[k]);
}
}
