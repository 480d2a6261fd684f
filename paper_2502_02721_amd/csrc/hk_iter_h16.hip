// Instantiations of the single-barrier blur kernel for 16-bit bases
// (bfloat16 and IEEE binary16) with FP32 operator data: the reduced-precision
// storage tier.  Arithmetic stays FP64; only the stored basis is rounded.
#include "hk_device.hpp"
#include "hk_blur.hpp"

namespace hk {

template <typename TB, int SK>
static const void* bptr(int ept)
{
    if (ept <= 1) return (const void*)&blur_iterate_kernel<TB, float, SK, 1>;
    if (ept <= 2) return (const void*)&blur_iterate_kernel<TB, float, SK, 2>;
    return (const void*)&blur_iterate_kernel<TB, float, SK, 4>;
}

// tb: 2 = bfloat16, 3 = binary16
const void* select_blur_h16(int tb, int sketch, int ept)
{
    if (tb == 2) return sketch == SK_GAUSS ? bptr<__bf16, SK_GAUSS>(ept) : bptr<__bf16, SK_SPARSE>(ept);
    if (tb == 3) return sketch == SK_GAUSS ? bptr<_Float16, SK_GAUSS>(ept) : bptr<_Float16, SK_SPARSE>(ept);
    return nullptr;
}

}  // namespace hk
