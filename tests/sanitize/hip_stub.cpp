// A CPU-only stand-in for the HIP runtime calls the library's host code
// makes, so that code (argument checks, tuning table, batch preparation,
// the serving runtime's scheduler) can run under AddressSanitizer,
// UndefinedBehaviorSanitizer and ThreadSanitizer on a machine with no GPU.
// Test infrastructure only: it is linked into the sanitizer test programs,
// never into the library.
//
// Semantics: every stream operation completes at once, in the calling
// thread (a copy is a memcpy on host memory, an event is complete as soon as
// it is recorded, elapsed times are 0).  "Device" memory is host memory.
// Graph capture is not supported (capture calls fail), so graph plans take
// their error paths.
#include <hip/hip_runtime_api.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>

namespace {
struct StubStream {
  int flags;
};
struct StubEvent {
  std::atomic<int> recorded{0};
};
}  // namespace

extern "C" {

hipError_t hipGetDevice(int* dev) {
  if (!dev) return hipErrorInvalidValue;
  *dev = 0;
  return hipSuccess;
}

hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  if (!p) return hipErrorInvalidValue;
  memset(p, 0, sizeof *p);
  strcpy(p->gcnArchName, "stub");
  return hipSuccess;
}

hipError_t hipRuntimeGetVersion(int* v) {
  if (!v) return hipErrorInvalidValue;
  *v = 1;
  return hipSuccess;
}

hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int flags) {
  if (!s) return hipErrorInvalidValue;
  *s = (hipStream_t) new StubStream{(int)flags};
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
  delete (StubStream*)s;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }

hipError_t hipEventCreate(hipEvent_t* e) {
  if (!e) return hipErrorInvalidValue;
  *e = (hipEvent_t) new StubEvent;
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) { return hipEventCreate(e); }

hipError_t hipEventDestroy(hipEvent_t e) {
  delete (StubEvent*)e;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  if (!e) return hipErrorInvalidValue;
  ((StubEvent*)e)->recorded.store(1);
  return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e) {
  if (!e) return hipErrorInvalidValue;
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (!ms || !a || !b) return hipErrorInvalidValue;
  *ms = 0.f;
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t bytes) {
  if (!p) return hipErrorInvalidValue;
  *p = malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) { return hipMalloc(p, bytes); }
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned int) {
  if (!d || !h) return hipErrorInvalidValue;
  *d = h;
  return hipSuccess;
}
hipError_t hipHostFree(void* p) { return hipFree(p); }

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  if (bytes && (!dst || !src)) return hipErrorInvalidValue;
  if (bytes) memcpy(dst, src, bytes);
  return hipSuccess;
}

// graphs: capture is not supported here
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  if (g) *g = nullptr;
  return hipErrorNotSupported;
}
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphExecUpdate(hipGraphExec_t, hipGraph_t, hipGraphNode_t*, hipGraphExecUpdateResult*) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphGetNodes(hipGraph_t, hipGraphNode_t*, size_t* n) {
  if (n) *n = 0;
  return hipErrorNotSupported;
}
hipError_t hipGraphNodeGetType(hipGraphNode_t, hipGraphNodeType*) { return hipErrorNotSupported; }
hipError_t hipGraphKernelNodeGetParams(hipGraphNode_t, hipKernelNodeParams*) { return hipErrorNotSupported; }

}  // extern "C"
