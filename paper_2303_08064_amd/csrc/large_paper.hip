// Launchers of the paper's default network (hidden 128 x 4, K = 8 with the
// selection output, the encoded input; FP32 and BF16), in a translation
// unit of their own. The kernels are in large.hpp.
#include "large.hpp"

namespace nasg {

NASG_LARGE_LAUNCHERS(paper, NASG_FOR_EACH_LARGE_NET_PAPER, NASG_FOR_EACH_STREAMED_QUERY_PAPER)

}  // namespace nasg
