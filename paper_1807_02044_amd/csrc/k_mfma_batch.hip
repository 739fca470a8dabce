// k_mfma_batch.hip - batched-plan launches of the matrix-core tile (tile code
// in mfma_tile.h).
#include "mfma_tile.h"

namespace fbs {

hipError_t launch_mfma_batch(const BatchClass& bc, hipStream_t s)
{
    return dispatch<BatchLauncher>(bc.r, bc.ch, bc.nw, bc, s);
}

int mfma_batch_blocks_per_cu(int r, int ch, int nw, int lds_bytes, bool co)
{
    int blocks = 0;
    if (dispatch<BatchOccupancy>(r, ch, nw, lds_bytes, co, &blocks) != hipSuccess) return 1;
    return blocks > 0 ? blocks : 1;
}

bool mfma_use_co(int D, int nb) { return use_co(D, nb); }

}  // namespace fbs
