// The exact path's kernels as one translation unit: the pair loop, the
// triangle pass, the per-node sums and the per-seed formulation, and the
// persistent batch kernel that runs all of them from one launch (it calls the
// same device code, which therefore has to be compiled together with it).
#include "exact/pairs.hip"
#include "exact/triangles.hip"
#include "exact/seed.hip"
#include "exact/batch_persist.hip"
