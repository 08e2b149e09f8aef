// Digit-pass kernels for uint64_t coordinates and uint64_t values (one translation unit per type
// pair so that the library builds in parallel).
#include "kernels_impl.h"

namespace qsd {

hipError_t digit_launch_u64_u64(const DigitArgs& a, int r, int items, hipStream_t s) {
    using CT = uint64_t;
    using VT = uint64_t;
    switch (r) {
        case 1: return digit_r<1, CT, VT>(a, items, s);
        case 2: return digit_r<2, CT, VT>(a, items, s);
        case 3: return digit_r<3, CT, VT>(a, items, s);
        case 4: return digit_r<4, CT, VT>(a, items, s);
        case 5: return digit_r<5, CT, VT>(a, items, s);
        case 6: return digit_r<6, CT, VT>(a, items, s);
        case 7: return digit_r<7, CT, VT>(a, items, s);
        case 8: return digit_r<8, CT, VT>(a, items, s);
    }
    return hipErrorInvalidValue;
}


}  // namespace qsd
