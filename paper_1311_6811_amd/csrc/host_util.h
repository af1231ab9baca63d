// Host-side helpers shared by the C ABI implementation files (not part of the ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>

#include "psfs_internal.h"

namespace psfs {
namespace host {

int fail(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
bool aligned(const void *p, size_t a);
bool finite_all(const float *v, int n);
int check_device();
int64_t padded_pixels(int width, int height);
size_t align256(size_t x);

// Autotuner cache (tune_cache.hip): $PSFS_AUTOTUNE_CACHE, else
// $HOME/.cache/psfs/autotune.json; callers hold tune_cache_mutex() around
// a read-modify-write.
std::string tune_cache_path();
std::mutex &tune_cache_mutex();
std::map<std::string, int> read_tune_cache(const std::string &path);
void write_tune_cache(const std::string &path, const std::map<std::string, int> &m);

}  // namespace host
}  // namespace psfs

#define PSFS_GUARD_BEGIN try {
#define PSFS_GUARD_END                                                                              \
    }                                                                                               \
    catch (const std::bad_alloc &) { return psfs::host::fail(PSFS_E_RANGE, "out of host memory"); } \
    catch (...) { return psfs::host::fail(PSFS_E_ARG, "unexpected exception"); }
