// vkt_internal.h -- declarations shared by the libvkt translation units.
//
// Nothing here is part of the public C interface (include/vkt.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/vkt.h"

namespace vkt {

// Number of bytes of one cell of a format.
inline int cell_bytes(vktDataFormat f)
{
    return f == vktDataFormatUInt8 ? 1 : (f == vktDataFormatUInt16 ? 2 : 4);
}

// Divisor-by-multiplication constants for an unsigned 32-bit divisor d >= 1
// (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Fig. 4.1): for every 32-bit n,
//   t = umulhi(m, n);  n / d == (t + ((n - t) >> sh1)) >> sh2.
struct UDiv {
    uint32_t m;
    uint32_t sh1;
    uint32_t sh2;
};
UDiv make_udiv(uint32_t d);

// Everything one single-volume ApplyFilter launch needs.
struct FilterJob {
    const void* src;
    void* dst;
    int32_t X, Y, Z;
    int32_t mode;            // vktAddressMode
    vktDataFormat fmt;       // format of src and dst
    int32_t k;
    const float* wf;         // device, k^3 float weights (float path)
    const int32_t* wi;       // device, k^3 int weights (integer path)
    bool int_filter;         // weights are integers with divisor D
    bool int_acc;            // integer accumulation (integer cells, int weights)
    int32_t D;
    UDiv div2D;              // for 2*D
    float inv_D;             // 1/D for float outputs of integer filters
    bool vec_store;          // dst rows can take 16-B-aligned vector stores
    float wscale;            // 2^s with max|w| * 2^s in [2^14, 2^15) (fp16 splitting)
};

// Kernel launchers (return the launch status).
hipError_t launch_fill(void* dst, int cell_bytes, int64_t n_cells,
                       uint32_t raw_bits, hipStream_t s);
hipError_t launch_fill_range(void* dst, int cell_bytes, int32_t X, int32_t Y,
                             const int32_t first[3], const int32_t last[3],
                             uint32_t raw_bits, hipStream_t s);
hipError_t launch_filter_valu(const FilterJob& j, hipStream_t s);
// Matrix-core path for float-weight filters with k >= 5.  six_products
// selects the 6-product bf16 split for float32 volumes (else 3 products).
hipError_t launch_filter_mfma(const FilterJob& j, bool six_products, hipStream_t s);

}  // namespace vkt
