// host_common.hpp -- host-side declarations of the library that need no HIP
// headers: the compiled kernel shapes, error reporting and the tuning
// tables and their cache file (tuning.cpp).  Plain C++, so that the cache
// reader and writer also build with an ordinary host compiler.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "phgrms.h"

namespace phg {

// A compiled kernel shape: passes per launch, rows per wave, waves per
// workgroup.  The tile is 256 columns wide (64 lanes x 4 pixels).
struct KernelShape {
  int T;
  int rows;
  int waves;
  int track;   // one-pass shapes: 1 keeps change maps (rows that cannot
               // change are copied through untested); 2 also leaves tiles
               // and rows that cannot change untouched from the third pass
               // on (the destination already holds them)
};
extern const KernelShape kShapes[];
extern const int kNumShapes;

// Set the calling thread's message (phgrms_last_error) and return `code`.
int fail(int code, const char* fmt, ...);

// Tuning is kept per beta and image size class: < 2^20, < 2^24, >= 2^24 pixels.
constexpr int kSizeClasses = 3;

// Both shape tables, as one value (tuning.cpp reads and writes them).
struct TuneTables {
  int fused[PHGRMS_BETA_MAX + 1][kSizeClasses];
  int batch[PHGRMS_BETA_MAX + 1][kSizeClasses];
};

// Read a tuning cache into t (entries the file does not name keep t's
// values); nothing changes on error.  PHGRMS_ENOTFOUND if there is no file.
int read_tuning_file(const char* path, TuneTables& t);
// Write t as a tuning cache, keeping the other keys of a valid existing file.
int write_tuning_file(const char* path, const TuneTables& t);

}  // namespace phg
