// Map / fixup kernels for 5-node episodes (all counter variants).
#include "fe_map.h"

namespace fe {
void launch_map_n5(bool exact, int dcls, const MapGroup &g, hipStream_t s, bool fix)
{
    map_dispatch_n<5>(exact, dcls, g, s, fix);
}
void launch_persist_n5(bool exact, int dcls, const BatchDev &b, int grid, const int *ctiles,
                       int nct, hipStream_t s, bool fix)
{
    persist_dispatch_n<5>(exact, dcls, b, grid, ctiles, nct, s, fix);
}
void launch_resume_n5(bool exact, int dcls, const MapGroup &g, int from, int *count_io,
                      int *last_io, hipStream_t s)
{
    resume_dispatch_n<5>(exact, dcls, g, from, count_io, last_io, s);
}
void launch_deep_n5(const DeepArgs &a, hipStream_t s) { deep_n<5>(a, s); }
}  // namespace fe
