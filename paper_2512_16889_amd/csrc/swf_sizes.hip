// Instantiation of the pass kernels for one group of FFT lengths and one
// precision.  Compiled several times with SWF_REAL and SWF_GROUP set by the
// build, so the (many, fully unrolled) kernels compile in parallel.
#include "swf_kernels.h"
#include "swf_reduce.h"

#ifndef SWF_REAL
#error "SWF_REAL must be float or double"
#endif
#ifndef SWF_GROUP
#error "SWF_GROUP must be set"
#endif

namespace swf {

#define SWF_CAT2(a, b) a##b
#define SWF_CAT(a, b) SWF_CAT2(a, b)
#define SWF_SIZE_FN(N) SWF_CAT(SWF_CAT(SWF_CAT(size_kernels_, SWF_TAG), _), N)
#define SWF_DEFINE(N)                                                  \
    const SizeKernels* SWF_SIZE_FN(N)() {                              \
        static const SizeKernels k = make_size_kernels<SWF_REAL, N>(); \
        return &k;                                                     \
    }

#if SWF_GROUP == 0
SWF_DEFINE(16)
SWF_DEFINE(32)
SWF_DEFINE(64)
SWF_DEFINE(128)
#elif SWF_GROUP == 7
SWF_DEFINE(48)
SWF_DEFINE(96)
SWF_DEFINE(192)
#elif SWF_GROUP == 8
SWF_DEFINE(40)
SWF_DEFINE(80)
SWF_DEFINE(160)
#elif SWF_GROUP == 1
SWF_DEFINE(256)
#elif SWF_GROUP == 2
SWF_DEFINE(512)
#elif SWF_GROUP == 3
SWF_DEFINE(1024)
#elif SWF_GROUP == 4
SWF_DEFINE(384)
#elif SWF_GROUP == 5
SWF_DEFINE(768)
#elif SWF_GROUP == 6
SWF_DEFINE(320)
#endif

}  // namespace swf
