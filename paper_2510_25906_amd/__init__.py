"""MI355X-native hybrid Linear / CWENOZ / MUSCL finite-volume reconstruction."""
