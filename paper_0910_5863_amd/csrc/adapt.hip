// placeholder replaced by the batched LOBPCG implementation
#include "adapt.h"

namespace bddc {
AdaptResult run_adapt(Problem &P, Solver &S, AdaptState &st, double tau) {
  (void)P; (void)S; (void)st; (void)tau;
  throw StateError("adaptivity is not built yet");
}
}  // namespace bddc
