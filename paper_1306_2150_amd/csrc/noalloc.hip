// The orthonormal sine transform without any device allocation, for callers
// that cannot allocate (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// Every device buffer the transform needs beyond the caller's input and
// output -- the sine tables of the grid size, the column descriptors of a
// launch, the split-K partial sums and the int8 slice records -- lives in one
// file-scope device array, `scratch`, of NA_SCRATCH_BYTES.  Each GPU the
// library runs on holds its own copy of it until the process ends.  Host code
// never uses the array's name as an address: the first call on a device looks
// up that device's copy with hipGetSymbolAddress and keeps the pointer.
//
// Every call on one GPU shares that GPU's array and overwrites what the last
// call left there; the call returns after its work completed, so calls from
// one host thread never overlap, but calls that overlap on one GPU (from
// several host threads, or while an earlier call's stream is still being
// captured) race.  The kernels are those of lrp_sine_transform, fed with the
// same host-built tables, so the results are the same bits.
#include <mutex>

#include "host.h"

namespace lrp {
namespace {

constexpr size_t NA_TAB_BYTES = (size_t)2 << 20;       // sine tables (<= 1.05 MB at n = 32767)
constexpr size_t NA_COLS = 1024;                        // column descriptors per launch
constexpr size_t NA_COLS_BYTES = (size_t)64 << 10;
constexpr size_t NA_PART_BYTES = (size_t)14 << 20;      // split-K partial sums
constexpr size_t NA_WORK_BYTES = (size_t)64 << 20;      // int8 slice records
constexpr size_t NA_SCRATCH_BYTES = NA_TAB_BYTES + NA_COLS_BYTES + NA_PART_BYTES + NA_WORK_BYTES;
static_assert(NA_COLS * sizeof(DstCol) <= NA_COLS_BYTES, "descriptor region");

__device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];

constexpr int NA_MAX_DEVICES = 64;
struct DeviceScratch {
  char *ptr = nullptr;   // this device's copy of `scratch` (device address)
  int tab_n = 0;         // grid size whose tables the copy holds (0: none)
};
DeviceScratch g_dev[NA_MAX_DEVICES];
std::mutex g_mu;
// host staging of the tables and descriptors (static: nothing is allocated)
char g_htab[NA_TAB_BYTES];
DstCol g_hcols[NA_COLS];

}  // namespace
}  // namespace lrp

using namespace lrp;

extern "C" lrp_status lrp_sine_transform_noalloc(int64_t n, int32_t ncols,
                                                 const double *src, int64_t lds,
                                                 double *dst, int64_t ldd, int32_t prec,
                                                 void *stream) {
  if (n < 1 || n > LRP_MAX_N || ncols < 0) return LRP_EINVAL;
  if (!transform_prec_ok(prec, (int)n)) return LRP_EINVAL;
  if (sine_table_bytes((int)n) > NA_TAB_BYTES) return LRP_EINVAL;
  // int8: the slice records of at least one column must fit
  const size_t col_work = dst_i8_work_bytes((int)n, 1);
  if (prec == LRP_PREC_INT8 && col_work > NA_WORK_BYTES) return LRP_EINVAL;
  if (ncols == 0) return LRP_OK;
  if (!src || !dst || lds < n || ldd < n) return LRP_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAX_DEVICES) return LRP_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch &ds = g_dev[dev];
  if (!ds.ptr) {
    // this device's copy of the array, looked up once with the device current
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LRP_EDEVICE;
    ds.ptr = (char *)p;
  }
  char *tab = ds.ptr;
  DstCol *dcols = (DstCol *)(ds.ptr + NA_TAB_BYTES);
  double *partial = (double *)(ds.ptr + NA_TAB_BYTES + NA_COLS_BYTES);
  void *work = ds.ptr + NA_TAB_BYTES + NA_COLS_BYTES + NA_PART_BYTES;
  // the previous call on this device returned after its work completed, so
  // the tables and descriptors may be rewritten now
  if (ds.tab_n != (int)n) {
    build_sine_table((int)n, g_htab);
    ds.tab_n = 0;
    if (hipMemcpyAsync(tab, g_htab, sine_table_bytes((int)n), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return LRP_EDEVICE;
    ds.tab_n = (int)n;
  }
  // columns per launch: the descriptor region, and for int8 the records
  size_t chunk = NA_COLS;
  if (prec == LRP_PREC_INT8) chunk = std::min(chunk, NA_WORK_BYTES / col_work);
  for (int c0 = 0; c0 < ncols; c0 += (int)chunk) {
    const int cnt = (int)std::min<size_t>(chunk, (size_t)(ncols - c0));
    for (int c = 0; c < cnt; ++c)
      g_hcols[c] = {src + (long)(c0 + c) * lds, dst + (long)(c0 + c) * ldd, -1, 0};
    if (hipMemcpyAsync(dcols, g_hcols, sizeof(DstCol) * cnt, hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return LRP_EDEVICE;
    if (launch_dst(prec, (int)n, tab, dcols, cnt, nullptr, partial, NA_PART_BYTES / 8, work,
                   NA_WORK_BYTES, st) != hipSuccess)
      return LRP_EDEVICE;
    // the descriptors' host staging is rewritten by the next chunk
    if (hipStreamSynchronize(st) != hipSuccess) return LRP_EDEVICE;
  }
  return LRP_OK;
}
