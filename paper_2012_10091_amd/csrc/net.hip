// Learned convolutional prolongation (placeholder until the kernels land).
#include "common.hpp"

namespace menkf {

hipError_t launch_net_prolong(const Plan &p, const void *dc, void *xf, const void *xprev, const menkf_net *net,
                              int fallback, void *ws, hipStream_t s) {
    (void)p; (void)dc; (void)xf; (void)xprev; (void)net; (void)fallback; (void)ws; (void)s;
    return hipErrorNotSupported;
}

}  // namespace menkf
