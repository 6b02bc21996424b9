// Serving pool (continuous batching of solves).
#include "common.h"
