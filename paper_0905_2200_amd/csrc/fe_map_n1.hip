// Map / fixup kernels for 1-node episodes (all counter variants).
#include "fe_map.h"

namespace fe {
void launch_map_n1(bool exact, int dcls, const MapGroup &g, hipStream_t s, bool fix)
{
    map_dispatch_n<1>(exact, dcls, g, s, fix);
}
}  // namespace fe
