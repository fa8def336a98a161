// runtime.hpp -- internals shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>

namespace otkm {

int map_hip(hipError_t e);
int init_locked();                 // requires lib_mutex()
std::mutex &lib_mutex();
hipStream_t lib_stream();
int device_cus();
void *pool_get(int slot, size_t bytes, int *err);                      // requires lib_mutex()
void *stream_ws(hipStream_t s, int slot, size_t bytes, int *err);      // requires lib_mutex()
void stream_ws_free(hipStream_t s);                                    // requires lib_mutex()
int default_block(int n);
int schedule_block(int n);
void schedule_set_locked(int t64, int t256);    // requires lib_mutex()

}  // namespace otkm
