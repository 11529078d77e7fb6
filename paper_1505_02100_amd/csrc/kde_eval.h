// Density evaluation kernels of libkdeplugin (internal interface between the
// host runtime and kde_eval.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kde {
namespace eval {

// Points per tile: one per thread (FP64 plain); 4096 (FP32), runs of 32 points
// shared by two threads, or 8 sub-tiles of 512 points, two per thread.
constexpr int kTilePoints64 = 256;
constexpr int kTilePoints32 = 4096;

struct EvalArgs {
    const void* x;     // samples on the device
    int64_t n;
    int32_t dtype;     // 0: FP64, 1: FP32 samples
    int32_t prec;      // 0: FP64 plain, 1: FP32 pair arithmetic
    const double* y;   // evaluation points on the device
    int64_t m;
    double h;          // bandwidth
    double s;          // sqrt(log2(e) / 2) / h
    double norm;       // 1 / (n h sqrt(2 pi))
    int64_t W;         // columns per chunk (multiple of 16)
    int32_t n_rt;      // tiles of points: 256 (FP64 plain) or 4096 (FP32)
    int32_t n_cc;      // column chunks
    double* part;      // n_cc x m partial sums (n_cc > 1)
    double* out;       // m results on the device
    int32_t* flag;     // set to 1 when a non-finite sample or point is read
};

// Enqueue the evaluation (and the chunk reduction when n_cc > 1) on s.
hipError_t launch(const EvalArgs& a, hipStream_t s);

// Blocks of the evaluation kernel for precision prec that one CU holds at once.
hipError_t blocks_per_cu(int prec, int* out);

}  // namespace eval
}  // namespace kde
