// Serving loop of liblkmi (continuous batching over many camera streams).
#include "lk_runtime.h"
