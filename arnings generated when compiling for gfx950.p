hipError_t launch_zero(void* out, int64_t n, int io, hipStream_t s);
