// AMNF per-window kernels, 7x7 window, Gaussian kernel (AMNFG): single-image and
// persistent batch launchers (the tile function is in kern_amnfe.h).
#include "kern_amnfe.h"

namespace vf {

int launch_amnfe_w7g(int eval, const KParams& p, int blocks, void* stream) {
    return amnfe_launch_w<7, true>(eval, p, blocks, stream);
}

int launch_amnfe_batch_w7g(int eval, const BatchParams& bp, int num_cus, void* stream, bool probe) {
    return amnfe_batch_launch_w<7, true>(eval, bp, num_cus, stream, probe);
}

}  // namespace vf
