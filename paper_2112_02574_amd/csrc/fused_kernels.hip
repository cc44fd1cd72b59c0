// fused_kernels.hip -- storage / order dispatch of the fused-step launchers;
// the kernels themselves are instantiated in fused_inst.hip (one object per
// storage format and stencil order).
#include "fused_impl.h"

namespace scmc {

#define SCMC_FUSED_COMBOS(X)                                                 \
    X(StoreF32, 4) X(StoreF32, 6) X(StoreF16, 4) X(StoreF16, 6)            \
    X(StoreBF16, 4) X(StoreBF16, 6)
#define SCMC_EXTERN(S, O) extern template struct FusedOps<S, O>;
SCMC_FUSED_COMBOS(SCMC_EXTERN)
#undef SCMC_EXTERN

template <class F> static bool with_ops(const StepKey &k, F &&fn) {
    if (k.dim != 3 || (k.order != 4 && k.order != 6) || k.big) return false;
    auto go = [&](auto stv) {
        using ST = decltype(stv);
        if (k.order == 4) return fn(FusedOps<ST, 4>{});
        return fn(FusedOps<ST, 6>{});
    };
    switch (k.storage) {
        case ST_F32: return go(StoreF32{});
        case ST_F16: return go(StoreF16{});
        case ST_BF16: return go(StoreBF16{});
    }
    return false;
}

bool fused_supported(const StepKey &k, const int *tile) {
    if (k.node) return false;  // node storage runs in the moment two-pass only
    return with_ops(k, [&](auto ops) { return decltype(ops)::supported(k, tile); });
}

hipError_t launch_fused(const StepKey &k, const Member &m, const void *src,
                        void *dst, const int *tile, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    with_ops(k, [&](auto ops) {
        err = decltype(ops)::launch(k, m, src, dst, tile, st);
        return true;
    });
    return err;
}

bool node_fused(const StepKey &k, const int *tile, NodeLaunch *node,
                const Member &m) {
    return with_ops(k, [&](auto ops) { return decltype(ops)::node(k, tile, node, m); });
}

hipError_t launch_batch_fused(const StepKey &k, const Member *d_members,
                              const Tile *d_tiles, int ntiles, const void *src,
                              void *dst, const int *tile, int grid,
                              hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    with_ops(k, [&](auto ops) {
        err = decltype(ops)::launch_batch(k, d_members, d_tiles, ntiles, src, dst,
                                          tile, grid, st);
        return true;
    });
    return err;
}

bool node_batch_fused(const StepKey &k, const int *tile, int grid,
                      NodeLaunch *node) {
    return with_ops(k, [&](auto ops) {
        return decltype(ops)::node_batch(k, tile, grid, node);
    });
}

}  // namespace scmc
