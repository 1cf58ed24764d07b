// Fused red-black sweeps (one HBM pass per sweep, optionally two sweeps per
// pass).  Placeholder: no fused variant is available yet, the solver uses the
// per-colour kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace isis {

template <class T, class M>
inline bool fused_supported(int) { return false; }

// Kernel launches made for `count` sweeps with temporal block tb.
inline int fused_launches(int count, int tb) { return (count + tb - 1) / tb; }

template <class T, class M>
inline int launch_fused_sweeps(const M&, int, double, T*, T*, const T*, const T*, int, int,
                               hipStream_t, char*)
{
    return -5;
}

}  // namespace isis
