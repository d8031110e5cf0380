// Device-resident join index (internal layout behind relnn_index).
#pragma once

#include <vector>

#include "common.hpp"

struct relnn_index {
  int device = 0;
  int k = 0;
  int64_t E = 0;             // joined tuples
  int64_t G = 0;             // groups (distinct head keys)
  int32_t* group_keys = nullptr;   // [G] ascending
  int32_t* offsets = nullptr;      // [G+1]
  int32_t* link_row = nullptr;     // [E] link row (or path number) per tuple
  int32_t* tuple_group = nullptr;  // [E] group number per tuple
  int32_t* rows = nullptr;         // [k*E] atom-major joined rows
  bool has_bwd = false;
  int64_t n_rows[RELNN_MAX_ATOMS] = {0, 0, 0, 0};
  bool atom_fd[RELNN_MAX_ATOMS] = {};     // atom's FK is a function of the head key
  bool atom_gk[RELNN_MAX_ATOMS] = {};     // atom's FK is the group column: one joined row per group
  // Transpose CSR of atom j (backward): tuples sorted by joined row.
  int32_t* t_off[RELNN_MAX_ATOMS] = {};   // [n_rows+1]
  int32_t* t_row[RELNN_MAX_ATOMS] = {};   // [E] joined row, ascending
  int32_t* t_pos[RELNN_MAX_ATOMS] = {};   // [E] canonical tuple position
  int32_t* t_grp[RELNN_MAX_ATOMS] = {};   // [E] group of that tuple
  // Its non-empty rows as segments: t_seg[E] segment of each position,
  // t_segoff[nseg+1], t_segrow[nseg] the row of each segment.
  int64_t t_nseg[RELNN_MAX_ATOMS] = {0, 0, 0, 0};
  int32_t* t_seg[RELNN_MAX_ATOMS] = {};
  int32_t* t_segoff[RELNN_MAX_ATOMS] = {};
  int32_t* t_segrow[RELNN_MAX_ATOMS] = {};
  int64_t dev_bytes = 0;
  std::vector<void*> allocs;

  template <class T>
  T* alloc(int64_t n) {
    void* p = nullptr;
    size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      relnn::set_error("index allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      throw relnn::Fail{RELNN_E_OOM};
    }
    allocs.push_back(p);
    dev_bytes += (int64_t)bytes;
    return static_cast<T*>(p);
  }
  ~relnn_index() {
    for (void* p : allocs) (void)hipFree(p);
  }
};
