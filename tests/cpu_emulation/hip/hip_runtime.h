#pragma once
#include "../hip_shim.h"
