/* Sizes and field offsets of the C-ABI structs that the Python binding
   mirrors with ctypes, printed as "name size offset..." lines (compiled by
   itself with gcc; the header is plain C). */
#include <stddef.h>
#include <stdio.h>

#include "../include/hsma.h"

#define F(T, f) printf(" %s=%zu", #f, offsetof(T, f))

int main(void) {
    printf("hsma_plan_desc %zu", sizeof(hsma_plan_desc));
    F(hsma_plan_desc, L); F(hsma_plan_desc, bc); F(hsma_plan_desc, p); F(hsma_plan_desc, M);
    F(hsma_plan_desc, K); F(hsma_plan_desc, R); F(hsma_plan_desc, precision); F(hsma_plan_desc, seed);
    F(hsma_plan_desc, near_mode); F(hsma_plan_desc, dipole_mode); F(hsma_plan_desc, dr);
    F(hsma_plan_desc, far_mode); F(hsma_plan_desc, gamma); F(hsma_plan_desc, far_shells);
    F(hsma_plan_desc, tree_order); F(hsma_plan_desc, tree_min_n);
    printf("\nhsma_plan_info_t %zu", sizeof(hsma_plan_info_t));
    F(hsma_plan_info_t, n_basis); F(hsma_plan_info_t, n_unknowns); F(hsma_plan_info_t, K);
    F(hsma_plan_info_t, n_check); F(hsma_plan_info_t, M_eff); F(hsma_plan_info_t, F1);
    F(hsma_plan_info_t, F2); F(hsma_plan_info_t, R0); F(hsma_plan_info_t, Rs);
    F(hsma_plan_info_t, precision); F(hsma_plan_info_t, bc); F(hsma_plan_info_t, bytes_resident);
    F(hsma_plan_info_t, near_mode); F(hsma_plan_info_t, max_images_per_source);
    F(hsma_plan_info_t, dipole_mode); F(hsma_plan_info_t, dr); F(hsma_plan_info_t, far_mode);
    F(hsma_plan_info_t, gamma); F(hsma_plan_info_t, far_shells); F(hsma_plan_info_t, tree_order);
    F(hsma_plan_info_t, tree_min_n);
    printf("\n");
    return 0;
}
