#include "hpa_internal.h"
