"""MI355X-native SPOCK Chambolle-Pock step library (arXiv:2505.12078)."""
