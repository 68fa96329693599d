// Shows that the host sanitizer harness catches the mistake it is there for:
// an asynchronous device-to-host copy into a stack variable of a function that
// returns before the stream is synchronised.  Built against the stand-in HIP
// runtime only (test infrastructure); the copy lands when the caller later
// synchronises, after the frame is gone.
#include <hip/hip_runtime_api.h>

#include <cstdio>

static void __attribute__((noinline)) returns_early(const int* dev, hipStream_t s) {
  int flag = 0;
  (void)hipMemcpyAsync(&flag, dev, sizeof(int), hipMemcpyDeviceToHost, s);
  // missing: hipStreamSynchronize(s) before flag goes out of scope
}

int main() {
  int* dev = nullptr;
  if (hipMalloc((void**)&dev, sizeof(int)) != hipSuccess) return 2;
  (void)hipMemset(dev, 0, sizeof(int));
  hipStream_t s = nullptr;
  (void)hipStreamCreateWithFlags(&s, 0);
  returns_early(dev, s);
  (void)hipStreamSynchronize(s);  // the late copy happens here
  std::printf("late copy not detected\n");
  return 0;
}
