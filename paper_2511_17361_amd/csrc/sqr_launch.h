// Workspace layout and cross-file launch helpers (host side).
#pragma once

#include "sqr_internal.h"

namespace sqr {

// Caller workspace, carved in this order (each part 256-byte aligned):
//   desc      device copy of the batch description (written by a kernel)
//   queue     2 x 8 per-XCD work counters (forward, backward), 128 B apart
//   boxes     [total_prims] packed neighbourhood boxes (index build)
//   partials  the index build's scratch: scan partial sums and the binning of
//             the primitives by voxel tile (index_scratch_bytes)
//   rec       [total_prims x REC] prepared primitive records
//   lgp       [total_prims x CP] logits padded to the compiled class width
//   acc       [total_prims x VP] backward gradient accumulators
//   lcount    2 ints: labelled pixels (semantic, depth) of the fused loss
//   lpart     [total_tiles x 2] per-tile loss partial sums
struct WsLayout {
    BatchDesc* desc;
    int* queue;
    int4* boxes;
    int64_t* partials;
    float* rec;
    float* lgp;
    float* acc;
    int* lcount;
    float* lpart;
};

int acc_row(int CP);
int scan_parts(const GridDev& g);
// bytes of the index build's own scratch (scan partials and tile binning)
size_t index_scratch_bytes(const GridDev& g, const BatchDesc& d);
WsLayout carve_ws(void* ws, const GridDev& g, const BatchDesc& d);
void put_desc(const BatchDesc& d, BatchDesc* dst, hipStream_t st);
void launch_index_kernels(const GridDev& g, const BatchDesc& d, const BatchDesc* desc_dev, const BatchIO& io,
                          int4* boxes, void* scratch, hipStream_t st);

}  // namespace sqr
