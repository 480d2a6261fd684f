// Instantiations of the persistent basis-iteration kernel for FP32 bases and FP32 operator data.
#include "hk_device.hpp"
#include "hk_blur.hpp"

namespace hk {

template <int OP, int SK, int EPT>
static const void* ptr()
{
    return (const void*)&iterate_kernel<float, float, OP, SK, EPT>;
}

template <int OP, int SK>
static const void* by_ept(int ept)
{
    if (ept <= 1) return ptr<OP, SK, 1>();
    if (ept <= 2) return ptr<OP, SK, 2>();
    if (ept <= 4) return ptr<OP, SK, 4>();
    return nullptr;
}

const void* select_iterate_f32(int op, int sketch, int ept)
{
    if (op == OP_BLUR) return sketch == SK_GAUSS ? by_ept<OP_BLUR, SK_GAUSS>(ept) : by_ept<OP_BLUR, SK_SPARSE>(ept);
    return sketch == SK_GAUSS ? by_ept<OP_CSR, SK_GAUSS>(ept) : by_ept<OP_CSR, SK_SPARSE>(ept);
}

template <int SK, int EPT>
static const void* bptr()
{
    return (const void*)&blur_iterate_kernel<float, float, SK, EPT>;
}

const void* select_blur_f32(int sketch, int ept)
{
    if (sketch == SK_GAUSS) return ept <= 1 ? bptr<SK_GAUSS, 1>() : ept <= 2 ? bptr<SK_GAUSS, 2>() : bptr<SK_GAUSS, 4>();
    return ept <= 1 ? bptr<SK_SPARSE, 1>() : ept <= 2 ? bptr<SK_SPARSE, 2>() : bptr<SK_SPARSE, 4>();
}

}  // namespace hk
