// device_types.h -- the HIP runtime and fixed-width integer types, both in
// the ahead-of-time build and when the device code is compiled at run time
// with hipRTC (which has no system headers and keeps these types in its own
// namespace).
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
using __hip_internal::int8_t;
using __hip_internal::int16_t;
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint8_t;
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif
