// Host-only stand-in for the HIP runtime, for bounds checks of kernel launches
// on a machine without a GPU (test infrastructure; never linked into the
// library).  Linked together with the library's own object files, it lets the
// real host code of the library run: every device allocation returns an address
// in a reserved range that is never dereferenced, every kernel launch is
// recorded (kernel name, grid, block, dynamic LDS, raw argument bytes) instead
// of executed, and copies from the device fill the host buffer with 0xFF bytes.
// The record is written to the file named by RBGS_LAUNCH_LOG, one line per
// event:
//   alloc <base> <bytes>
//   launch <mangled name> <gx> <gy> <gz> <bx> <by> <bz> <shmem> <nargs> <hex bytes of each arg>
//   copy <dst> <src> <bytes> <kind>
//   data <dst> <hex bytes>      (the bytes of a host -> device copy)
#include <cxxabi.h>
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <string>
#include <vector>

namespace {

FILE* log_file() {
  static FILE* f = nullptr;
  if (!f) {
    const char* p = getenv("RBGS_LAUNCH_LOG");
    f = fopen(p ? p : "launch_log.txt", "w");
  }
  return f;
}

std::map<const void*, std::string>& names() {
  static std::map<const void*, std::string> m;
  return m;
}

uint64_t next_addr = 0x100000000000ull;   // 16 TiB: outside any host mapping used here
std::map<uint64_t, uint64_t> live;          // base -> bytes

struct CallCfg {
  dim3 grid, block;
  size_t shmem;
  hipStream_t stream;
};
std::vector<CallCfg> cfg_stack;

// Sizes of the parameters of a demangled "name(T1, T2, ...)" signature.
std::vector<int> param_sizes(const std::string& dem) {
  std::vector<int> out;
  const size_t open = dem.find('(');
  const size_t close = dem.rfind(')');
  if (open == std::string::npos || close == std::string::npos || close <= open + 1) return out;
  std::string params = dem.substr(open + 1, close - open - 1);
  int depth = 0;
  std::string cur;
  auto flush = [&]() {
    std::string t = cur;
    while (!t.empty() && t[0] == ' ') t.erase(0, 1);
    int sz = 8;
    if (t.find('*') != std::string::npos || t.find('&') != std::string::npos) sz = 8;
    else if (t == "int" || t == "unsigned int" || t == "float") sz = 4;
    else if (t == "short" || t == "unsigned short") sz = 2;
    else if (t == "bool" || t == "char" || t == "unsigned char") sz = 1;
    out.push_back(sz);
    cur.clear();
  };
  for (char ch : params) {
    if (ch == '<' || ch == '(') ++depth;
    if (ch == '>' || ch == ')') --depth;
    if (ch == ',' && depth == 0) flush();
    else cur += ch;
  }
  flush();
  return out;
}

}  // namespace

extern "C" {

void** __hipRegisterFatBinary(const void*) {
  static void* dummy[4];
  return dummy;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void* hostFunction, char* deviceFunction, const char*,
                           unsigned int, uint3*, uint3*, dim3*, dim3*, int*) {
  names()[hostFunction] = deviceFunction;
}

// __device__ variables: their host shadow address -> size; a lookup of the
// device address is logged as an allocation of that size (once per variable).
std::map<const void*, size_t>& vars() {
  static std::map<const void*, size_t> m;
  return m;
}
std::map<const void*, uint64_t>& var_addr() {
  static std::map<const void*, uint64_t> m;
  return m;
}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  vars()[var] = size;
}

hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shmem, hipStream_t st) {
  cfg_stack.push_back({g, b, shmem, st});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* shmem, hipStream_t* st) {
  CallCfg c = cfg_stack.back();
  cfg_stack.pop_back();
  *g = c.grid;
  *b = c.block;
  *shmem = c.shmem;
  *st = c.stream;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void* fn, dim3 g, dim3 b, void** args, size_t shmem, hipStream_t) {
  const std::string& mangled = names()[fn];
  int status = 0;
  char* dem = abi::__cxa_demangle(mangled.c_str(), nullptr, nullptr, &status);
  std::vector<int> sizes = param_sizes(dem ? std::string(dem) : std::string());
  free(dem);
  FILE* f = log_file();
  fprintf(f, "launch %s %u %u %u %u %u %u %zu %zu", mangled.c_str(), g.x, g.y, g.z, b.x, b.y, b.z,
          shmem, sizes.size());
  for (size_t i = 0; i < sizes.size(); ++i) {
    unsigned char buf[8] = {0};
    memcpy(buf, args[i], sizes[i]);
    fprintf(f, " ");
    for (int j = 0; j < sizes[i]; ++j) fprintf(f, "%02x", buf[j]);
  }
  fprintf(f, "\n");
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t bytes) {
  const uint64_t base = next_addr;
  next_addr += ((bytes + 0xFFFFFull) & ~0xFFFFFull) + (1ull << 20);  // 1 MiB gap after each
  live[base] = bytes;
  *p = (void*)base;
  fprintf(log_file(), "alloc %llu %zu\n", (unsigned long long)base, bytes);
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  auto it = vars().find(symbol);
  if (it == vars().end()) return hipErrorInvalidSymbol;
  auto a = var_addr().find(symbol);
  if (a == var_addr().end()) {
    void* q = nullptr;
    hipMalloc(&q, it->second);
    a = var_addr().emplace(symbol, (uint64_t)q).first;
  }
  *p = (void*)a->second;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  live.erase((uint64_t)p);
  fprintf(log_file(), "free %llu\n", (unsigned long long)(uint64_t)p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
  *p = calloc(1, bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  free(p);
  return hipSuccess;
}

static hipError_t copy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  fprintf(log_file(), "copy %llu %llu %zu %d\n", (unsigned long long)(uint64_t)dst,
          (unsigned long long)(uint64_t)src, bytes, (int)kind);
  if (kind == hipMemcpyDeviceToHost) memset(dst, 0xFF, bytes);
  // host -> device uploads of up to 8 MiB (descriptor arrays): their bytes
  if (kind == hipMemcpyHostToDevice && bytes <= (8u << 20)) {
    FILE* f = log_file();
    fprintf(f, "data %llu ", (unsigned long long)(uint64_t)dst);
    const unsigned char* b = (const unsigned char*)src;
    for (size_t i = 0; i < bytes; ++i) fprintf(f, "%02x", b[i]);
    fprintf(f, "\n");
  }
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  return copy(dst, src, bytes, kind);
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t) {
  return copy(dst, src, bytes, kind);
}

hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t attr, int) {
  *v = attr == hipDeviceAttributeMultiprocessorCount ? 256
       : attr == hipDeviceAttributeWallClockRate    ? 100000
                                                    : 0;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock"; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  static char dummy[64];
  static int next = 1;
  *s = (hipStream_t)(dummy + (next++ % 64));
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t)malloc(16);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  free((void*)e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }

}  // extern "C"
