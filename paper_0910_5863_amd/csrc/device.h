// Device-resident state of one BDDC problem and the kernels that move data
// between the global vector, the substructure interfaces and the coarse space.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dense.h"
#include "host.h"

namespace bddc {

struct DevAlloc {
  void *(*alloc)(size_t, void *) = nullptr;
  void (*free)(void *, void *) = nullptr;
  void *user = nullptr;
  size_t held = 0;
  void *get(size_t bytes);
  void put(void *p, size_t bytes);
};

// Device buffer with its byte size (owned by the context's allocator).
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  template <class T>
  T *as() const {
    return reinterpret_cast<T *>(p);
  }
};

// Per (substructure, constrained glob) record for applying T / T^T.
struct GlobXf {
  int sub;
  int m, ng;
  int64_t trow_off;  // m x ng row-major in the trow and wmat pools
  int64_t pos_off;   // ng interface positions (absolute in the sum-nG stack)
  int64_t piv_off;   // m pivot positions (absolute)
  int64_t scr_off;   // m scratch values per vector
  int64_t scrS_off;  // m x nG(sub) scratch values for matrix transforms
};

// Precision-independent layout of one factorized problem.
struct Layout {
  int nsub = 0;
  int64_t n_glob = 0;
  std::vector<int> nI, nG, nr, np;
  std::vector<int64_t> offI, offG, offR, offP;         // vector stacks
  std::vector<int64_t> offGG, offRR, offRP, offPP;  // matrix pools
  int64_t sumI = 0, sumG = 0, sumR = 0, sumP = 0;
  int64_t sGG = 0, sRR = 0, sRP = 0, sPP = 0;
  int64_t n_gamma = 0;  // global interface dofs
  int64_t n_coarse = 0;
  int max_nI = 0, max_nG = 0, max_nr = 0, max_np = 0;
};

}  // namespace bddc
