// Host check of the mapping from the update step's status bits to C-ABI
// statuses (compiled by itself with g++; the header is HIP-free).
#include <cstdio>
#include <cstring>

#include "../paper_1806_04801_amd/csrc/result_status.h"

using namespace hsma;

static int fails = 0;

static void expect(int bits, hsma_status want) {
    const char* msg = nullptr;
    const hsma_status got = status_of_bits(bits, &msg);
    if (got != want || (want == HSMA_OK) != (msg == nullptr)) {
        printf("bits %d: got %d want %d\n", bits, (int)got, (int)want);
        ++fails;
    }
}

int main() {
    expect(0, HSMA_OK);
    expect(RS_BAD_INPUT, HSMA_E_INVALID);
    expect(RS_OUT_OF_BOX, HSMA_E_OUT_OF_BOX);
    expect(RS_NOT_NEUTRAL, HSMA_E_NOT_NEUTRAL);
    expect(RS_COINCIDENT, HSMA_E_COINCIDENT);
    expect(RS_NONFINITE, HSMA_E_NONFINITE);
    // an input error explains a non-finite result and takes precedence
    expect(RS_BAD_INPUT | RS_NONFINITE, HSMA_E_INVALID);
    expect(RS_COINCIDENT | RS_NONFINITE, HSMA_E_COINCIDENT);
    expect(RS_OUT_OF_BOX | RS_NOT_NEUTRAL, HSMA_E_OUT_OF_BOX);
    // every combination of bits maps to the status of its lowest bit
    const hsma_status order[] = {HSMA_E_INVALID, HSMA_E_OUT_OF_BOX, HSMA_E_NOT_NEUTRAL,
                                 HSMA_E_COINCIDENT, HSMA_E_NONFINITE};
    for (int bits = 1; bits < 32; ++bits) {
        int low = 0;
        while (!(bits & (1 << low))) ++low;
        expect(bits, order[low]);
    }
    const char* msg = nullptr;
    status_of_bits(RS_NONFINITE, &msg);
    if (msg == nullptr || strstr(msg, "non-finite") == nullptr) ++fails;
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
