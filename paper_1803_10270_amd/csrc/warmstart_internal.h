// Internal descriptors of the learned warm start (host side and kernels).
#pragma once
#include <stdint.h>

namespace cpws {

constexpr int NLAYER = 4;
constexpr int CH_IN = 3, CH_HID = 32;
constexpr int N_PARAMS = 3 * 32 * 5 + 32 + 2 * (32 * 32 * 5 + 32) + 32 * 5 + 1;   // 10977

// One convolution layer: parameter offset (natural order W[o][c][t] then b[o]), channel
// counts and their padded widths, and the BF16 matrix shapes of the forward product
// (NoPf x Kpf, k = t CiP + c) and of its adjoint (NoPb x Kpb, k = t CoP + o).
struct LayerDesc {
    int32_t off, Ci, Co, CiP, CoP, Kpf, NoPf, Kpb, NoPb;
};

inline LayerDesc layer_desc(int l) {
    static const int ci[NLAYER] = {CH_IN, CH_HID, CH_HID, CH_HID};
    static const int co[NLAYER] = {CH_HID, CH_HID, CH_HID, 1};
    LayerDesc L;
    int off = 0;
    for (int j = 0; j < l; ++j) off += co[j] * ci[j] * 5 + co[j];
    L.off = off;
    L.Ci = ci[l];
    L.Co = co[l];
    L.CiP = (ci[l] + 7) / 8 * 8;
    L.CoP = (co[l] + 7) / 8 * 8;
    L.Kpf = (5 * L.CiP + 31) / 32 * 32;
    L.NoPf = (L.Co + 15) / 16 * 16;
    L.Kpb = (5 * L.CoP + 31) / 32 * 32;
    L.NoPb = (L.Ci + 15) / 16 * 16;
    return L;
}

}  // namespace cpws
