// FFT-length dispatch: maps (precision, n) to the kernel table compiled for it.
#include "swf_kernels.h"
#include "swf_reduce.h"

namespace swf {

#define SWF_DECL(TAG, N) const SizeKernels* size_kernels_##TAG##_##N();
#define SWF_SIZES(X, TAG) X(TAG, 16) X(TAG, 32) X(TAG, 64) X(TAG, 128) X(TAG, 256) X(TAG, 512) X(TAG, 1024) \
    X(TAG, 48) X(TAG, 96) X(TAG, 192) X(TAG, 384) X(TAG, 768) X(TAG, 40) X(TAG, 80) X(TAG, 160) X(TAG, 320)
SWF_SIZES(SWF_DECL, f32)
SWF_SIZES(SWF_DECL, f64)

#define SWF_CASE(TAG, N) case N: return size_kernels_##TAG##_##N();

const SizeKernels* size_kernels(int fp64, int n) {
    if (fp64) {
        switch (n) { SWF_SIZES(SWF_CASE, f64) default: return nullptr; }
    }
    switch (n) { SWF_SIZES(SWF_CASE, f32) default: return nullptr; }
}

}  // namespace swf
