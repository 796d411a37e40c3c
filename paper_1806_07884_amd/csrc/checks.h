// Device-side index checks of the checked build (compiled with RBF_CHECKED).
//
// RBF_CHECK(P, cond) is true when cond holds.  In a checked build a false
// cond also records the check's place (source file id * 100000 + line) in the
// plan's check word, first failure wins, and the caller skips the access it
// guards; the C-ABI reads the word after the entry point's kernels and
// returns RBF_ERR_HIP naming the place.  In a normal build the checks are the
// constant true and compile to nothing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The check word alone, for kernels that take no plan view.
struct CheckWord {
  int32_t* check;
};

#ifdef RBF_CHECKED
#define RBF_CHECKED_BUILD 1
#define RBF_CHECK(P, cond)                                                         \
  ((cond) ? true                                                                   \
          : ((P).check ? (atomicCAS((P).check, 0, RBF_CHECK_FILE * 100000 + __LINE__), \
                          false)                                                   \
                       : false))
#else
#define RBF_CHECKED_BUILD 0
#define RBF_CHECK(P, cond) true
#endif
