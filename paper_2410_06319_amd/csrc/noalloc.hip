// ls_qr_r_noalloc: Algorithm 1's QR with its scratch in a static device array.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops).  The working copy of Y, the Householder
// scalars, the T factors and the flag word of the QR live in `scratch`, a
// file-scope device array of LS_NOALLOC_SCRATCH_BYTES that every GPU the
// library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// the device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and is used everywhere the memory is needed.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace {

using namespace ls;

static __device__ __align__(256) char scratch[LS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDev = 64;
struct ScratchTable {
  std::mutex mu;
  char* ptr[kMaxDev] = {};
};
ScratchTable& scratch_table() {
  static ScratchTable t;
  return t;
}

// The device address of `scratch` on the current device (resolved on the
// first call there).
int scratch_ptr(char** out) {
  int dev = 0;
  LS_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return LS_E_UNSUPPORTED;
  ScratchTable& t = scratch_table();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.ptr[dev]) {
    void* p = nullptr;
    LS_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return LS_E_HIP;
    t.ptr[dev] = static_cast<char*>(p);
  }
  *out = t.ptr[dev];
  return LS_OK;
}

// The flag word starts at zero: a one-thread kernel clears it (no memset node
// for callers that capture the stream).
__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

}  // namespace

extern "C" int ls_qr_r_noalloc(int64_t s, int64_t ncols, ls_prec_t u_qr, double* Y, int64_t ldy, double* R,
                               int64_t ldr, void* stream) {
  if (!Y || !R || ncols < 1 || s < ncols || ldy < s || ldr < ncols) return LS_E_ARG;
  if (u_qr != LS_FP32 && u_qr != LS_FP64) return LS_E_UNSUPPORTED;
  // the flag word takes the first 256 bytes, the QR's workspace the rest
  const size_t need = 256 + qr_workspace(s, ncols, u_qr);
  if (need > (size_t)LS_NOALLOC_SCRATCH_BYTES) return LS_E_WORKSPACE;
  char* base = nullptr;
  LS_TRY(scratch_ptr(&base));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* flag = reinterpret_cast<int*>(base);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, flag);
  LS_HIP_TRY(hipGetLastError());
  LS_TRY(qr_run(s, ncols, u_qr, Y, ldy, R, ldr, base + 256, (size_t)LS_NOALLOC_SCRATCH_BYTES - 256, flag, ncols,
                st));
  int h = 0;
  LS_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  LS_HIP_TRY(hipStreamSynchronize(st));
  return qr_flag_status(h);
}
