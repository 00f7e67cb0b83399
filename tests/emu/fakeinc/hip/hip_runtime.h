#pragma once
#include "../../emu_hip.h"
