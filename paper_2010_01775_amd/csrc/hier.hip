// Adaptive octree build (placeholder until the sort-based build lands).
#include "npg_internal.h"

extern "C" int npg_build_hierarchy(npg_ctx *ctx, const float *pos_dev, uint64_t n,
                                   const npg_hier_params *params, uint32_t *perm_dev,
                                   uint32_t *leaf_of_dev, uint32_t *leaf_off_dev,
                                   uint64_t *leaf_key_dev, uint8_t *leaf_depth_dev,
                                   uint32_t max_leaves, uint32_t *n_leaves_out, void *stream) {
  (void)pos_dev; (void)n; (void)params; (void)perm_dev; (void)leaf_of_dev; (void)leaf_off_dev;
  (void)leaf_key_dev; (void)leaf_depth_dev; (void)max_leaves; (void)n_leaves_out; (void)stream;
  if (!ctx) return NPG_E_ARG;
  return npg_fail(ctx, NPG_E_ARG, "build_hierarchy: not available in this build");
}
