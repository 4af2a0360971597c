// AMNF per-window kernels (exponential and Gaussian kernel): the 3x3 and 5x5
// instantiations and the launchers over all window sizes (the 7x7 kernels are
// instantiated in kern_amnfe_w7.hip and kern_amnfe_w7g.hip; the tile function
// is in kern_amnfe.h).
#include "kern_amnfe.h"

namespace vf {

int launch_amnfe_w7(int eval, const KParams& p, int blocks, void* stream);
int launch_amnfe_w7g(int eval, const KParams& p, int blocks, void* stream);
int launch_amnfe_batch_w7(int eval, const BatchParams& bp, int num_cus, void* stream, bool probe);
int launch_amnfe_batch_w7g(int eval, const BatchParams& bp, int num_cus, void* stream, bool probe);

int launch_amnfe(int filter, int window, int eval, const KParams& p, int blocks, void* stream) {
    const bool g = filter == VF_FILTER_AMNFG;
    switch (window) {
    case 3: return g ? amnfe_launch_w<3, true>(eval, p, blocks, stream) : amnfe_launch_w<3, false>(eval, p, blocks, stream);
    case 5: return g ? amnfe_launch_w<5, true>(eval, p, blocks, stream) : amnfe_launch_w<5, false>(eval, p, blocks, stream);
    case 7: return g ? launch_amnfe_w7g(eval, p, blocks, stream) : launch_amnfe_w7(eval, p, blocks, stream);
    }
    return -1;
}

// Persistent batch launch (see launch_persistent); -1 when no kernel matches.
int launch_amnfe_batch(int filter, int window, int eval, const BatchParams& bp, int num_cus, void* stream,
                       bool probe) {
    const bool g = filter == VF_FILTER_AMNFG;
    switch (window) {
    case 3:
        return g ? amnfe_batch_launch_w<3, true>(eval, bp, num_cus, stream, probe)
                 : amnfe_batch_launch_w<3, false>(eval, bp, num_cus, stream, probe);
    case 5:
        return g ? amnfe_batch_launch_w<5, true>(eval, bp, num_cus, stream, probe)
                 : amnfe_batch_launch_w<5, false>(eval, bp, num_cus, stream, probe);
    case 7:
        return g ? launch_amnfe_batch_w7g(eval, bp, num_cus, stream, probe)
                 : launch_amnfe_batch_w7(eval, bp, num_cus, stream, probe);
    }
    return -1;
}

}  // namespace vf
