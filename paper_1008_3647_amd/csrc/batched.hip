// Batched persistent solver (placeholder translation unit; filled in below).
#include "ufg_internal.h"
