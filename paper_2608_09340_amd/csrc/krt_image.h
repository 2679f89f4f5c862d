// krt_image.h -- launch of the imaging pass whose duration is taken by HIP
// events that the dispatch itself records at the kernel's start and end, so
// the figure excludes the host's launch latency (an event recorded on an idle
// stream before the launch completes before the kernel's packet arrives).
#pragma once
#include <hip/hip_runtime.h>

#include "krt_kernels.h"

namespace krt {

// start / stop: created events, or null for an untimed launch
hipError_t launch_image_timed(const ImageParams &Q, hipStream_t s, hipEvent_t start, hipEvent_t stop);

}  // namespace krt
