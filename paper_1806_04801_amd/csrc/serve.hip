// Batched serving executor (continuous batching of energy/force requests).
#include "hsma_internal.h"
