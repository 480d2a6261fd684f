// Instantiations of the persistent basis-iteration kernel for FP64 bases and FP64 operator data.
#include "hk_device.hpp"
#include "hk_blur.hpp"

namespace hk {

template <int OP, int SK, int EPT>
static const void* ptr(int samp)
{
    return samp ? (const void*)&iterate_kernel<double, double, OP, SK, EPT, true>
                : (const void*)&iterate_kernel<double, double, OP, SK, EPT, false>;
}

template <int OP, int SK>
static const void* by_ept(int ept, int samp)
{
    if (ept <= 1) return ptr<OP, SK, 1>(samp);
    if (ept <= 2) return ptr<OP, SK, 2>(samp);
    if (ept <= 4) return ptr<OP, SK, 4>(samp);
    return nullptr;
}

const void* select_iterate_f64(int op, int sketch, int ept, int samp)
{
    if (op == OP_BLUR)
        return sketch == SK_GAUSS ? by_ept<OP_BLUR, SK_GAUSS>(ept, samp) : by_ept<OP_BLUR, SK_SPARSE>(ept, samp);
    return sketch == SK_GAUSS ? by_ept<OP_CSR, SK_GAUSS>(ept, samp) : by_ept<OP_CSR, SK_SPARSE>(ept, samp);
}

template <int SK, int EPT>
static const void* bptr()
{
    return (const void*)&blur_iterate_kernel<double, double, SK, EPT>;
}

const void* select_blur_f64(int sketch, int ept)
{
    if (sketch == SK_GAUSS) return ept <= 1 ? bptr<SK_GAUSS, 1>() : ept <= 2 ? bptr<SK_GAUSS, 2>() : bptr<SK_GAUSS, 4>();
    return ept <= 1 ? bptr<SK_SPARSE, 1>() : ept <= 2 ? bptr<SK_SPARSE, 2>() : bptr<SK_SPARSE, 4>();
}

}  // namespace hk
